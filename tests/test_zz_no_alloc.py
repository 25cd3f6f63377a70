"""etc_solve_static (setup + solve + K_eff in the library's static scratch
array, for callers that cannot allocate) against the allocating entry
points etc_setup / etc_solve / etc_keff / etc_get_solution on the same
input.  Both run the same kernels with the same launch shapes, so pass
counts agree exactly and K and the solution to rounding (1e-13 relative).

Two static calls run back to back, the second on a smaller grid, so the
second finds the first call's contents in the shared array.
"""

import numpy as np
import pytest

import rvegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

etc = pytest.importorskip("paper_2404_02433_amd")


def allocating(x, axis, precision, rtol):
    plan = etc.etc_setup(x, axis, precision=precision, rtol=rtol)
    out = etc.etc_solve(plan)
    out.update(etc.etc_keff(plan))
    p = etc.etc_get_solution(plan)
    torch.cuda.synchronize()
    plan.close()
    return out, p


@pytest.mark.parametrize("precision,dtype", [("fp64", np.float64), ("mixed", np.float32)])
def test_static_scratch_matches_allocating_entry_points(precision, dtype):
    cases = [((40, 36, 44), 0, 11), ((20, 26, 18), 1, 12)]   # second call smaller
    for shape, axis, seed in cases:
        print(f"no-alloc {precision}: shape {shape} axis {axis} seed {seed}", flush=True)
        kap = rvegen.random_two_phase(shape, seed=seed, kappa=(1.0, 100.0)).astype(dtype)
        x = torch.as_tensor(kap, device="cuda:0")
        ref, p_ref = allocating(x, axis, precision, 1e-8)
        p = torch.full(x.shape, float("nan"), dtype=torch.float64, device=x.device)
        got = etc.etc_solve_static(x, axis, precision=precision, rtol=1e-8, out=p)
        torch.cuda.synchronize()
        print(f"no-alloc {precision}: K={got['keff']:.15g} ref={ref['keff']:.15g} iters {got['iters']}/{ref['iters']}",
              flush=True)
        assert got["status"] == "ok" and ref["status"] == "ok"
        assert got["iters"] == ref["iters"]
        assert abs(got["keff"] - ref["keff"]) <= 1e-13 * abs(ref["keff"])
        assert abs(got["k_in"] - ref["k_in"]) <= 1e-13 * abs(ref["k_in"])
        assert torch.isfinite(p).all()
        assert (p - p_ref).abs().max().item() <= 1e-13 * p_ref.abs().max().item()


def test_static_scratch_rejects_a_grid_beyond_its_size():
    x = torch.ones((128, 128, 128), dtype=torch.float64, device="cuda:0")
    with pytest.raises(etc.EtcError) as e:
        etc.etc_solve_static(x, 0)
    assert e.value.status == -6
