"""The allocation-free stepping entry point (dg_rk_step_noalloc) against
dg_rk_step, through the C ABI: the same kernels on the library's per-GPU
scratch instead of a caller workspace, so the states must agree bitwise.
Two calls in a row, the second on a smaller mesh (the scratch keeps the
first call's contents), then a mesh too large for the scratch."""
import numpy as np
import pytest

import synthetic
from helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIMS = [320, 256, 256, 256, 320]
NORM = [1.0, 0.0, 0.0, 0.0, synthetic.TGV_ENERGY_LEVEL, 0.01, 1, 1, 1, 1, 0, 0, 0, 0, 0, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3]


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_11571_amd import binding
    binding.lib()
    return binding


def _perturbed(B, m, seed):
    q = m.field()
    B.dg_init_tgv(m, q)
    g = torch.Generator(device="cpu").manual_seed(seed)
    q[1:4] += 0.01 * torch.randn(q[1:4].shape, generator=g, dtype=torch.float64).cuda()
    return q


def _both(B, N, P, Re, steps, model=None, seed=0):
    m = B.Mesh(N, P, Re)
    q0 = _perturbed(B, m, seed)
    dt = B.dg_stable_dt(m, q0)
    q_ref, k_ref = q0.clone(), m.field(0.0)
    B.dg_rk_step(m, q_ref, k_ref, dt, steps, model=model)
    q, k = q0.clone(), m.field(0.0)
    B.dg_rk_step_noalloc(m, q, k, dt, steps, model=model)
    torch.cuda.synchronize()
    return q_ref.cpu().numpy(), q.cpu().numpy(), k_ref.cpu().numpy(), k.cpu().numpy()


def test_noalloc_equals_workspace_stepping_two_calls(B):
    model = B.Model(DIMS, B.pack_params(synthetic.mlp_init(DIMS, seed=0)), NORM, train=False)
    say("no-alloc call 1: 16^3 P = 3 with the network, 2 steps")
    q_ref, q, k_ref, k = _both(B, 16, 3, 200.0, 2, model=model, seed=1)
    assert np.isfinite(q).all()
    assert np.array_equal(q, q_ref) and np.array_equal(k, k_ref)
    say("no-alloc call 2: 4^3 P = 6 plain, 3 steps")
    q_ref, q, k_ref, k = _both(B, 4, 6, 1600.0, 3, seed=2)
    assert np.isfinite(q).all()
    assert np.array_equal(q, q_ref) and np.array_equal(k, k_ref)


def test_noalloc_rejects_meshes_beyond_the_scratch(B):
    say("no-alloc size limit")
    m = B.Mesh(16, 6, 1600.0)
    assert m.ws_bytes > (96 << 20)
    q, k = m.field(1.0), m.field(0.0)
    with pytest.raises(B.DGError) as ei:
        B.dg_rk_step_noalloc(m, q, k, 1e-4, 1)
    assert ei.value.code == B.DG_ENOSPC
    assert "no-alloc scratch" in str(ei.value)
