"""Host-side checks of the autograd wrappers (no GPU work is started):
coupled_run only differentiates frictionless, non-sub-cycled, dynamic DEM
steps, and says so before it allocates anything."""
import pytest
import torch

import workloads as W


@pytest.mark.parametrize("bad", [dict(mu_f=0.3, k_t=1e-3), dict(theta_r=0.01), dict(n_sub=2),
                                 dict(kinematic=True)])
def test_coupled_run_rejects_what_its_adjoint_does_not_cover(bad):
    from paper_1901_09745_amd.autograd import coupled_run
    z = torch.zeros(1, 3, dtype=torch.float64)
    with pytest.raises(ValueError):
        coupled_run(z, z, z, torch.zeros(9), W.LatticeSpec(q=9, nx=8, ny=8),
                    torch.ones(1, dtype=torch.float64), W.DemSpec(**bad), 3)
