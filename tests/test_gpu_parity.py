"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Element-by-element comparisons on seeded inputs at sizes the oracle finishes
in seconds, chosen to span several tiles and ragged tails (b not a multiple
of 64, a not a multiple of 4, k chunks, FFT lengths with radices 2-16, 3 and
5, and the O(N^2) route for odd or prime lengths).

Tolerances: float64 results within a few ulps times the problem's own
rounding growth (DCTs of length N lose ~log2(N) ulps; the tridiagonal
solves' condition number is O(nL^2)); mixed-precision results against the
float64 oracle within the 1e-5 relative K_eff target.
"""

import math

import numpy as np
import pytest

import rvegen
from oracle import etc_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

etc = pytest.importorskip("paper_2404_02433_amd")


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def lognormal(shape, seed, sigma=1.0):
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal(shape))


# ------------------------------------------------------------------ operator
@pytest.mark.parametrize("shape,axis", [((37, 29, 70), 0), ((12, 17, 9), 1), ((20, 8, 33), 2), ((2, 1, 1), 0)])
def test_operator_matches_oracle_fp64(shape, axis):
    kap = lognormal(shape, seed=sum(shape))
    plan = etc.etc_setup(dev(kap), axis)
    pb = O.make_problem(kap, axis)
    x = np.random.default_rng(1).standard_normal(pb.shape)
    y, d = etc.etc_apply_A(plan, dev(x), want_dot=True)
    ref = O.apply_A(pb, x)
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err
    assert abs(d - float(np.vdot(x, ref))) < 1e-12 * abs(float(np.vdot(x, ref)))
    plan.close()


# float32 lines of 66 take 64-wide stencil tiles (one ragged), lines of 300
# 128-wide ones (the last 44 wide)
@pytest.mark.parametrize("shape", [(33, 21, 66), (9, 21, 300)])
def test_operator_matches_oracle_mixed(shape):
    kap = rvegen.random_two_phase(shape, seed=4, kappa=(1.0, 100.0))
    plan = etc.etc_setup(dev(kap), 0, precision="mixed")
    pb = O.make_problem(kap, 0)
    x = np.random.default_rng(2).standard_normal(pb.shape).astype(np.float32)
    y, d = etc.etc_apply_A(plan, dev(x, torch.float32), want_dot=True)
    ref = O.apply_A(pb, x.astype(np.float64))
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 2e-6, err
    # w . q from the float32 products summed in float64 per tile
    dref = float(np.vdot(x.astype(np.float64), ref))
    assert abs(d - dref) < 1e-5 * abs(dref), (d, dref)
    plan.close()


# ------------------------------------------------------------ preconditioner
PRECOND_SHAPES = [
    (16, 32, 64),    # radices 16, 16x2
    (10, 48, 40),    # 48 -> M=24 (8x3); 40 -> M=20 (4x5)
    (9, 7, 12),      # odd a: O(N^2) route; 12 -> M=6 (2x3)
    (8, 1, 5),       # a of length 1; b odd
    (6, 80, 2),      # 80 -> M=40 (8x5); b=2 -> M=1
    (5, 96, 160),    # 96 -> M=48 (16x3); 160 -> M=80 (16x5)
    (64, 128, 34),   # 128 -> 16x4; 34 -> M=17 prime: O(N^2) route; nL=64: 32 partitions of 2
    (33, 16, 16),    # nL not a multiple of the partition length
    (96, 8, 12),     # exact partitions of 3 rows
    (128, 5, 7),     # exact partitions of 4 rows
    (160, 6, 10),    # exact partitions of 5 rows
    (256, 4, 16),    # exact partitions of 8 rows
    (3, 256, 160),   # compile-time column length 256, row length 160
    (2, 48, 512),    # compile-time column length 48, row length 512
    (300, 3, 5),     # ragged partitions (no exact variant), 10 rows each
    (4, 500, 6),     # 500 -> M=250 (2x5x5x5): 16 columns would need 4 radix-5 butterflies per thread
    (3, 486, 4),     # 486 -> M=243 (3^5): 16 columns would need 6 radix-3 butterflies per thread
]


@pytest.mark.parametrize("shape", PRECOND_SHAPES)
def test_preconditioner_matches_oracle_fp64(shape):
    kap = lognormal(shape, seed=3 + sum(shape), sigma=0.7)
    plan = etc.etc_setup(dev(kap), 0)
    pb = O.make_problem(kap, 0)
    kref = O.kref_mid(pb)
    r = np.random.default_rng(5).standard_normal(pb.shape)
    z, rz = etc.etc_apply_Minv(plan, dev(r), want_dot=True)
    ref = O.apply_Aref_inv(r, kref)
    err = np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-11, err
    assert abs(rz - float(np.vdot(r, ref))) < 1e-10 * abs(float(np.vdot(r, ref)))
    plan.close()


# Every compiled tridiagonal block shape (modes x partitions per line) on
# load axes that hit its exact partition lengths and its ragged (guarded)
# ones; b = 37 leaves a partial tile of modes for every shape.
THOMAS_LENGTHS = {
    8: [10, 20, 33, 48, 64, 96, 100, 128],
    16: [48, 100, 160, 200, 256],
    32: [64, 96, 100, 128, 160, 200, 256, 300, 512, 700, 1500, 2048],
}
THOMAS_SHAPES = {"fp64": [(32, 8), (16, 16), (32, 16), (16, 32)],
                 "mixed": [(32, 8), (16, 16), (64, 8), (32, 16), (32, 32)]}
# The float32 32-row partition variant (load axes 513-1024 in the mixed form)
# faulted on its first run with no cause found in its indexing; it is no
# longer compiled and the mixed form refuses load axes above 512.
_NO_F32_LONG = pytest.mark.skip(reason="float32 guarded partitions of more than 16 rows are switched off (the "
                                       "32x32 variant of up to 32 rows faulted; mixed-form load axes stop at 512)")
# exact partitions of more than 16 rows: 32x16 at 512 (32 rows), 32x8 at 160
# and 256 (20 and 32 rows)
_EXACT_LONG = {(32, 16): [512], (32, 8): [160, 256]}
THOMAS_CASES = [pytest.param(prec, tb, p, nl, marks=_NO_F32_LONG) if prec == "mixed" and nl > 512
                else (prec, tb, p, nl)
                for prec, shapes in THOMAS_SHAPES.items() for tb, p in shapes
                for nl in THOMAS_LENGTHS[p] + _EXACT_LONG.get((tb, p), [])]


@pytest.mark.parametrize("precision,tb,parts,nl", THOMAS_CASES)
def test_preconditioner_every_tridiagonal_shape(precision, tb, parts, nl):
    shape = (nl, 5, 37)
    kap = lognormal(shape, seed=nl + tb + parts, sigma=0.7)
    mixed = precision == "mixed"
    tdt = torch.float32 if mixed else torch.float64
    print(f"tridiagonal {tb}x{parts} {precision} nL={nl}", flush=True)
    plan = etc.etc_setup(dev(kap, tdt), 0, precision=precision, thomas_shape=(tb, parts))
    assert etc.etc_launch_info(plan)["thomas_shape"] == (tb, parts)
    pb = O.make_problem(kap.astype(np.float32).astype(np.float64) if mixed else kap, 0)
    r = np.random.default_rng(nl).standard_normal(pb.shape)
    if mixed:
        r = r.astype(np.float32)
    z, rz = etc.etc_apply_Minv(plan, dev(r, tdt), want_dot=True)
    plan.close()
    ref = O.apply_Aref_inv(r.astype(np.float64), O.kref_mid(pb))
    err = np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()
    rz_ref = float(np.vdot(r.astype(np.float64), ref))
    assert err < (1e-5 if mixed else 1e-11), err
    assert abs(rz - rz_ref) < (1e-5 if mixed else 1e-10) * abs(rz_ref)


def test_tridiagonal_shape_that_does_not_hold_the_axis_is_rejected():
    kap = dev(lognormal((200, 4, 4), seed=1))
    for shape in ((32, 8), (7, 7), (32, 32)):
        with pytest.raises(RuntimeError):
            etc.etc_setup(kap, 0, thomas_shape=shape)  # (32, 32) is float32 only
    etc.etc_setup(kap, 0, thomas_shape=(16, 32)).close()
    for nl, want in ((64, (32, 8)), (128, (32, 8)), (150, (16, 16)), (160, (32, 8)), (200, (32, 16)),
                     (256, (32, 8)), (257, (16, 32)), (512, (32, 16))):
        plan = etc.etc_setup(dev(lognormal((nl, 4, 4), seed=2)), 0)
        assert etc.etc_launch_info(plan)["thomas_shape"] == want, nl
        plan.close()


# Run-time FFT lengths whose radix-3 or radix-5 stages bound the lines per
# block below 16 complex values per thread: rows of 300 (M=150), 270 (135),
# 200 (100) and 384 (192), columns of 500 (250) and 486 (243).
FFT_RADIX_BOUND = [(20, 6, 300), (12, 5, 270), (20, 6, 200), (20, 6, 384), (4, 500, 6), (3, 486, 4)]


@pytest.mark.parametrize("shape", [(96, 8, 12), (256, 4, 16), (3, 256, 160), (2, 48, 512), (300, 3, 5), (64, 6, 40),
                                   (33, 16, 16), (4, 128, 64), (5, 512, 32), (3, 512, 40), (2, 64, 160)]
                         + FFT_RADIX_BOUND)
def test_preconditioner_mixed_shapes(shape):
    """float32 storage: compile-time (one-instance plans: persistent column)
    kernels, exact and ragged tridiagonal partitions."""
    kap = lognormal(shape, seed=17 + sum(shape), sigma=0.7)
    plan = etc.etc_setup(dev(kap, torch.float32), 0, precision="mixed")
    pb = O.make_problem(kap.astype(np.float32).astype(np.float64), 0)
    r = np.random.default_rng(9).standard_normal(pb.shape).astype(np.float32)
    z = etc.etc_apply_Minv(plan, dev(r, torch.float32))
    ref = O.apply_Aref_inv(r.astype(np.float64), O.kref_mid(pb))
    err = np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-5, err
    plan.close()


def _five_smooth(m):
    for r in (2, 3, 5):
        while m % r == 0:
            m //= r
    return m == 1


# Every FFT-route length up to 640 (N even, N/2 with no prime factor above 5)
# and a few dense-route ones, as rows (64 lines: row blocks at their largest)
# and as columns (32 columns: column tiles at their widest).
FFT_SWEEP = [n for n in range(4, 641, 2) if _five_smooth(n // 2)] + [7, 34, 101, 257, 514]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("where", ["rows", "cols"])
def test_preconditioner_every_fft_length(precision, where):
    mixed = precision == "mixed"
    tdt = torch.float32 if mixed else torch.float64
    bad = []
    for n in FFT_SWEEP:
        shape = (8, 8, n) if where == "rows" else (2, n, 32)
        kap = lognormal(shape, seed=n, sigma=0.5)
        if mixed:
            kap = kap.astype(np.float32).astype(np.float64)
        plan = etc.etc_setup(dev(kap, tdt), 0, precision=precision)
        r = np.random.default_rng(n).standard_normal(shape)
        if mixed:
            r = r.astype(np.float32)
        z = etc.etc_apply_Minv(plan, dev(r, tdt))
        plan.close()
        pb = O.make_problem(kap, 0)
        ref = O.apply_Aref_inv(r.astype(np.float64), O.kref_mid(pb))
        err = np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()
        if not err < (1e-5 if mixed else 1e-11):
            bad.append((n, float(err)))
    print(f"{where} {precision}: {len(FFT_SWEEP)} lengths, failing {bad}", flush=True)
    assert not bad, bad


def test_preconditioner_mixed_close_to_oracle():
    shape = (32, 64, 96)
    kap = lognormal(shape, seed=8)
    plan = etc.etc_setup(dev(kap, torch.float32), 0, precision="mixed")
    pb = O.make_problem(kap.astype(np.float32).astype(np.float64), 0)
    r = np.random.default_rng(6).standard_normal(pb.shape).astype(np.float32)
    z = etc.etc_apply_Minv(plan, dev(r, torch.float32))
    ref = O.apply_Aref_inv(r.astype(np.float64), O.kref_mid(pb))
    err = np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-5, err
    plan.close()


# --------------------------------------------------------------------- solve
def test_spheres32_fp64_trajectory_and_keff():
    """32^3 two-phase RVE (12 spheres of radius 4, kappa 1/10), rtol 1e-10:
    same iteration count and residual history as the oracle's PCG and K_eff
    within 1e-9."""
    kap, info = rvegen.make_config("spheres32")
    ref = O.solve(kap, 0, rtol=1e-10)
    plan = etc.etc_setup(dev(kap), 0, rtol=1e-10)
    out = etc.etc_solve(plan)
    k = etc.etc_keff(plan, energy=True)
    assert out["status"] == "ok"
    assert abs(out["iters"] - ref["iters"]) <= 1
    assert abs(k["keff"] - ref["keff"]) <= 1e-9 * ref["keff"]
    assert abs(k["k_in"] - ref["k_in"]) <= 1e-9 * ref["keff"]
    assert abs(k["k_energy"] - ref["k_energy"]) <= 1e-9 * ref["keff"]
    hist = etc.etc_residual_history(plan)
    oh = ref["pcg"].history
    n = min(len(hist), len(oh), 12)
    np.testing.assert_allclose(hist[:n], oh[:n], rtol=1e-7)
    for i, v in enumerate(out["kref"]):
        assert abs(v - ref["kref"][O.FAMILIES[i]]) <= 1e-14 * v
    plan.close()


def test_mixed_keff_within_1e5_of_fp64_truth():
    kap, _ = rvegen.make_config("spheres32")
    truth = O.solve(kap, 0, rtol=1e-12)["keff"]
    for dt in (torch.float64, torch.float32):
        out = etc.solve(dev(kap, dt), 0, precision="mixed", rtol=1e-6)
        assert out["status"] == "ok"
        assert abs(out["keff"] - truth) <= 1e-5 * truth, (dt, out["keff"], truth)
        assert out["relres"] <= 1e-6


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_axes_and_solution_layout(axis):
    shape = (14, 11, 19)
    kap = rvegen.random_two_phase(shape, seed=10 + axis, kappa=(1.0, 20.0))
    ref = O.solve(kap, axis, p_in=2.0, p_out=-1.0, rtol=1e-11)
    plan = etc.etc_setup(dev(kap), axis, p_in=2.0, p_out=-1.0, rtol=1e-11)
    etc.etc_solve(plan)
    k = etc.etc_keff(plan)
    assert abs(k["keff"] - ref["keff"]) <= 1e-9 * ref["keff"]
    p = etc.etc_get_solution(plan).cpu().numpy()
    pref = O.decanonical(ref["pcg"].p, axis)
    assert np.abs(p - pref).max() < 1e-9
    plan.close()


@pytest.mark.parametrize("shape", [(2, 3, 4), (6, 1, 1), (5, 1, 7), (3, 2, 1), (2, 1, 1)])
def test_degenerate_shapes(shape):
    kap = rvegen.random_two_phase(shape, seed=1, kappa=(0.5, 4.0))
    ref = O.solve(kap, 0, rtol=1e-13)
    out = etc.solve(dev(kap), 0, rtol=1e-13)
    assert abs(out["keff"] - ref["keff"]) <= 1e-11 * ref["keff"]


def test_homogeneous_is_exact_in_one_pass():
    kap = np.full((24, 20, 18), 3.7)
    out = etc.solve(dev(kap), 0, rtol=1e-12, L=(2.0, 1.0, 0.5), p_in=5.0, p_out=1.0)
    assert out["iters"] == 1
    assert abs(out["keff"] - 3.7) < 1e-11


def test_laminates_on_gpu():
    layers = 10 ** np.random.default_rng(3).uniform(-2, 2, size=40)
    kap = rvegen.series_laminate((40, 16, 24), layers, 0)
    out = etc.solve(dev(kap), 0, rtol=1e-13)
    harm = len(layers) / np.sum(1 / layers)
    assert abs(out["keff"] - harm) < 1e-10 * harm
    plane = 10 ** np.random.default_rng(4).uniform(-2, 2, size=(16, 24))
    kap = rvegen.parallel_laminate((40, 16, 24), plane, 0)
    out = etc.solve(dev(kap), 0, rtol=1e-13)
    assert abs(out["keff"] - plane.mean()) < 1e-10 * plane.mean()


def test_invalid_conductivity_rejected():
    kap = np.ones((8, 8, 8))
    kap[3, 4, 5] = 0.0
    with pytest.raises(etc.EtcError) as e:
        etc.etc_setup(dev(kap), 0)
    assert e.value.status == -1
    kap[3, 4, 5] = np.nan
    with pytest.raises(etc.EtcError):
        etc.etc_setup(dev(kap), 0)


def test_iteration_cap_reports_not_converged():
    kap, _ = rvegen.make_config("spheres32")
    plan = etc.etc_setup(dev(kap), 0, rtol=1e-12, max_iter=3)
    out = etc.etc_solve(plan)
    assert out["status"] == "not_converged" and out["iters"] == 3
    ref = O.pcg(O.make_problem(kap, 0), rtol=1e-12, max_iter=3)
    k = etc.etc_keff(plan)
    assert abs(k["keff"] - O.keff(O.make_problem(kap, 0), ref.p)["out"]) < 1e-9
    plan.close()


def test_bitwise_deterministic():
    kap = lognormal((40, 36, 52), seed=12)
    outs = []
    for _ in range(2):
        plan = etc.etc_setup(dev(kap), 0, rtol=1e-9)
        etc.etc_solve(plan)
        outs.append(etc.etc_get_solution(plan).cpu().numpy())
        plan.close()
    assert np.array_equal(outs[0], outs[1])


def test_warm_start_resume():
    kap = lognormal((30, 28, 26), seed=13)
    plan = etc.etc_setup(dev(kap), 0, rtol=1e-3)
    etc.etc_solve(plan)
    p_mid = etc.etc_get_solution(plan)
    plan.close()
    plan = etc.etc_setup(dev(kap), 0, rtol=1e-10)
    out = etc.etc_solve(plan, p0=p_mid)
    k_resumed = etc.etc_keff(plan)["keff"]
    plan.close()
    direct = etc.solve(dev(kap), 0, rtol=1e-10)["keff"]
    assert out["status"] == "ok"
    assert abs(k_resumed - direct) < 1e-8 * direct


# ------------------------------------------------------------------ gradient
@pytest.mark.parametrize("axis,precision", [(0, "fp64"), (2, "fp64"), (1, "mixed")])
def test_adjoint_gradient_matches_oracle(axis, precision):
    """etc_grad (adjoint PCG + face-product kernel) against the oracle's
    dissipation-form gradient, which equals dK/dkappa at the exact solution."""
    shape = (18, 14, 22)
    kap = lognormal(shape, seed=31 + axis, sigma=0.8)
    rtol = 1e-12 if precision == "fp64" else 1e-7
    plan = etc.etc_setup(dev(kap), axis, p_in=1.5, p_out=0.5, rtol=rtol, precision=precision, want_grad=True)
    etc.etc_solve(plan)
    g = etc.etc_grad(plan).cpu().numpy()
    k_after = etc.etc_keff(plan)["keff"]
    pb = O.make_problem(kap, axis, p_in=1.5, p_out=0.5)
    ref = O.solve(kap, axis, p_in=1.5, p_out=0.5, rtol=1e-13)
    gref = O.decanonical(O.keff_gradient(pb, ref["pcg"].p), axis)
    tol = 1e-8 if precision == "fp64" else 1e-4
    assert np.abs(g - gref).max() <= tol * np.abs(gref).max()
    # the primal state survives the adjoint solve
    assert abs(k_after - ref["keff"]) <= (1e-9 if precision == "fp64" else 1e-5) * ref["keff"]
    plan.close()


def test_gradient_finite_differences_on_gpu():
    shape = (16, 12, 20)
    kap = lognormal(shape, seed=41, sigma=1.0)
    plan = etc.etc_setup(dev(kap), 0, rtol=1e-13, want_grad=True)
    etc.etc_solve(plan)
    g = etc.etc_grad(plan).cpu().numpy()
    plan.close()
    rng = np.random.default_rng(3)
    for _ in range(8):
        v = tuple(int(rng.integers(0, s)) for s in shape)
        d = 1e-4 * kap[v]
        vals = []
        for sgn in (1, -1):
            k2 = kap.copy()
            k2[v] += sgn * d
            vals.append(etc.solve(dev(k2), 0, rtol=1e-13)["keff"])
        fd = (vals[0] - vals[1]) / (2 * d)
        assert abs(fd - g[v]) <= 1e-6 * np.abs(g).max() + 1e-6 * abs(g[v]), (v, fd, g[v])


def test_autograd_function():
    kap = lognormal((12, 10, 14), seed=5)
    x = dev(kap).requires_grad_(True)
    k = etc.keff(x, 0, rtol=1e-12)
    (gx,) = torch.autograd.grad(3.0 * k, x)
    plan = etc.etc_setup(dev(kap), 0, rtol=1e-12, want_grad=True)
    etc.etc_solve(plan)
    g = etc.etc_grad(plan)
    # etc_grad_as: the same float64 gradient rounded once to float32
    assert torch.equal(etc.etc_grad(plan, torch.float32), g.to(torch.float32))
    plan.close()
    assert torch.allclose(gx, 3.0 * g, rtol=1e-10, atol=1e-14)
    # float32 kappa: the gradient comes back in kappa's dtype; without
    # requires_grad no adjoint solve runs and K is the same
    x32 = dev(kap, torch.float32).requires_grad_(True)
    (g32,) = torch.autograd.grad(etc.keff(x32, 0, rtol=1e-12), x32)
    assert g32.dtype == torch.float32 and g32.shape == x32.shape
    ref32 = etc.etc_setup(dev(kap, torch.float32), 0, rtol=1e-12, want_grad=True)
    etc.etc_solve(ref32)
    g_ref = etc.etc_grad(ref32, torch.float32)
    ref32.close()
    assert torch.equal(g32, g_ref)
    with torch.no_grad():
        assert abs(float(etc.keff(dev(kap), 0, rtol=1e-12)) - float(k)) <= 1e-14 * float(k)


def test_grad_requires_want_grad():
    kap = lognormal((8, 8, 8), seed=6)
    plan = etc.etc_setup(dev(kap), 0)
    etc.etc_solve(plan)
    with pytest.raises(etc.EtcError) as e:
        etc.etc_grad(plan)
    assert e.value.status == -5
    plan.close()


# ------------------------------------------- orthotropic kappa, sources, faces
from problems import smooth_problem  # noqa: E402


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [32, 64])
def test_smooth_orthotropic_table1_on_gpu(n, precision):
    """tab:smooth: L2 error of the TPFA solution of the smooth orthotropic
    problem (source term, Dirichlet data varying over the faces)."""
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "table1_smooth.json")) as f:
        t1 = json.load(f)
    comps, src, pin, pout, exact = smooth_problem(n)
    rtol = 1e-9 if precision == "fp64" else 1e-7
    plan = etc.etc_setup([dev(c) for c in comps], 2, precision=precision, rtol=rtol, L=(1.0, 1.0, 1.0),
                         source=dev(src), p_in_face=dev(pin), p_out_face=dev(pout))
    out = etc.etc_solve(plan)
    p = etc.etc_get_solution(plan).cpu().numpy()
    plan.close()
    err = math.sqrt(np.sum((p - exact) ** 2) / n ** 3)
    ref = t1["l2_error_rtol_1e-9"][t1["n"].index(n)]
    assert out["status"] == "ok"
    assert abs(err - ref) <= 0.006 * ref, (n, err, ref)
    if precision == "fp64":
        assert out["iters"] == t1["iters_rtol_1e-9"][t1["n"].index(n)]


def test_orthotropic_operator_and_solution_match_oracle():
    shape = (21, 17, 26)
    rng = np.random.default_rng(9)
    comps = [np.exp(0.6 * rng.standard_normal(shape)) for _ in range(3)]
    src = rng.standard_normal(shape)
    pin = 1.0 + 0.1 * rng.standard_normal((shape[0], shape[2]))
    pout = -0.5 + 0.1 * rng.standard_normal((shape[0], shape[2]))
    axis = 1
    pb = O.make_problem(None, axis, pin, pout, L=(2.0, 1.0, 1.5), components=comps, source=src)
    plan = etc.etc_setup([dev(c) for c in comps], axis, p_in=1.0, p_out=-0.5, rtol=1e-12, L=(2.0, 1.0, 1.5),
                         source=dev(src), p_in_face=dev(pin), p_out_face=dev(pout))
    x = rng.standard_normal(pb.shape)
    y = etc.etc_apply_A(plan, dev(x)).cpu().numpy()
    ref = O.apply_A(pb, x)
    assert np.abs(y - ref).max() < 1e-13 * np.abs(ref).max()
    z = etc.etc_apply_Minv(plan, dev(x)).cpu().numpy()
    zref = O.apply_Aref_inv(x, O.kref_mid(pb))
    assert np.abs(z - zref).max() < 1e-11 * np.abs(zref).max()
    etc.etc_solve(plan)
    p = etc.etc_get_solution(plan).cpu().numpy()
    pref = O.decanonical(O.pcg(pb, rtol=1e-13).p, axis)
    assert np.abs(p - pref).max() < 1e-9 * np.abs(pref).max()
    plan.close()


# ------------------------------------------------ preconditioner comparisons
def test_plain_cg_grows_with_grid_and_dct_pcg_does_not():
    """prop:cond: cond(A) ~ nL^2, so plain CG needs about twice the passes when
    the grid doubles; the DCT/Thomas preconditioner keeps the count flat.
    Both reach the same K_eff (center ball, kappa_inc = 10)."""
    its_cg, its_pcg = [], []
    for n in (32, 64, 128):
        kap = dev(rvegen.center_ball(n, 10.0))
        a = etc.solve(kap, 2, rtol=1e-8, precond="none", max_iter=20000)
        b = etc.solve(kap, 2, rtol=1e-8)
        assert a["status"] == "ok" and b["status"] == "ok"
        assert abs(a["keff"] - b["keff"]) < 1e-7 * b["keff"]
        its_cg.append(a["iters"])
        its_pcg.append(b["iters"])
    assert its_cg[1] > 1.6 * its_cg[0] and its_cg[2] > 1.6 * its_cg[1], its_cg
    assert max(its_pcg) - min(its_pcg) <= 6, its_pcg


def test_reference_parameter_modes_reach_the_same_keff():
    """'one' and 'mid' reference parameters change the pass count, not K_eff."""
    kap = dev(rvegen.center_ball(48, 1000.0))
    mid = etc.solve(kap, 2, rtol=1e-9)
    one = etc.solve(kap, 2, rtol=1e-9, kref="one")
    usr = etc.solve(kap, 2, rtol=1e-9, kref="user", kref_user=[2.0, 2.0, 2.0, 2.0, 2.0])
    for o in (one, usr):
        assert o["status"] == "ok"
        assert abs(o["keff"] - mid["keff"]) < 1e-7 * mid["keff"]
    assert one["kref"] == [1.0] * 5


# ----------------------------------------------------------------- batches
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_individual_solves(precision):
    """A batch of same-size RVEs in one plan: every instance reaches the K_eff
    of its own solve; per-instance exit tests (the instances converge after
    different pass counts)."""
    n = 24
    kaps = [np.exp(s * np.random.default_rng(100 + i).standard_normal((n, n, n))) for i, s in
            enumerate([0.2, 0.6, 1.0, 1.4, 0.1])]
    batch = dev(np.stack(kaps))
    rtol = 1e-10 if precision == "fp64" else 1e-6
    out = etc.solve_batch(batch, 0, precision=precision, rtol=rtol)
    assert all(st == "ok" for st in out["status"])
    assert len(set(out["iters"])) > 1
    for i, k in enumerate(kaps):
        ref = O.solve(k, 0, rtol=1e-12)
        tol = 1e-8 if precision == "fp64" else 1e-5
        assert abs(out["keff"][i] - ref["keff"]) <= tol * ref["keff"], (i, out["keff"][i], ref["keff"])
        single = etc.solve(dev(k), 0, precision=precision, rtol=rtol)
        assert out["iters"][i] == single["iters"]
        if precision == "fp64":
            assert out["keff"][i] == single["keff"]   # same reductions, same order


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_with_persistent_column_kernels(precision):
    """A batch whose column length has compile-time kernels (64) and whole
    column tiles runs the persistent column kernels until an instance
    converges, then the gated ones: every instance still reaches its own
    solve's K_eff and the oracle's."""
    shape = (16, 64, 64)
    kaps = [np.exp(s * np.random.default_rng(300 + i).standard_normal(shape)) for i, s in enumerate([0.1, 0.8, 1.5])]
    rtol = 1e-10 if precision == "fp64" else 1e-6
    out = etc.solve_batch(dev(np.stack(kaps)), 0, precision=precision, rtol=rtol)
    assert all(st == "ok" for st in out["status"])
    assert len(set(out["iters"])) > 1
    for i, k in enumerate(kaps):
        ref = O.solve(k, 0, rtol=1e-12)
        tol = 1e-8 if precision == "fp64" else 1e-5
        assert abs(out["keff"][i] - ref["keff"]) <= tol * ref["keff"], (i, out["keff"][i], ref["keff"])
        single = etc.solve(dev(k), 0, precision=precision, rtol=rtol)
        assert abs(out["iters"][i] - single["iters"]) <= 1
        assert abs(out["keff"][i] - single["keff"]) <= tol * ref["keff"]


def test_batch_solution_and_gradient_layout():
    n = (10, 12, 14)
    kaps = np.stack([np.exp(0.5 * np.random.default_rng(7 + i).standard_normal(n)) for i in range(3)])
    plan = etc.etc_setup_batch(dev(kaps), 2, rtol=1e-12, want_grad=True)
    etc.etc_solve(plan)
    p = etc.etc_get_solution(plan).cpu().numpy()
    g = etc.etc_grad(plan).cpu().numpy()
    plan.close()
    for i in range(3):
        ref = O.solve(kaps[i], 2, rtol=1e-13)
        assert np.abs(p[i] - O.decanonical(ref["pcg"].p, 2)).max() < 1e-9
        gref = O.decanonical(O.keff_gradient(ref["problem"], ref["pcg"].p), 2)
        assert np.abs(g[i] - gref).max() < 1e-8 * np.abs(gref).max()


# ------------------------------------------------------------- HIP graphs
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_equals_eager(precision):
    """use_graph replays captured passes: every solve of a plan (the graph is
    captured once and replayed many times, with eager work and host
    synchronisation between the replays) gives the eager path's iterates bit
    for bit, and the adjoint solve captures a graph of its own."""
    kap = lognormal((26, 30, 44), seed=77, sigma=1.2)
    rtol = 1e-10 if precision == "fp64" else 1e-6
    eager = etc.etc_setup(dev(kap), 0, rtol=rtol, precision=precision, want_grad=True)
    e_out = etc.etc_solve(eager)
    e_p = etc.etc_get_solution(eager).cpu().numpy()
    e_k = etc.etc_keff(eager)["keff"]
    e_g = etc.etc_grad(eager).cpu().numpy()
    eager.close()
    plan = etc.etc_setup(dev(kap), 0, rtol=rtol, precision=precision, want_grad=True, use_graph=True)
    for rep in range(3):
        out = etc.etc_solve(plan)
        assert out["iters"] == e_out["iters"] and out["status"] == "ok", rep
        assert np.array_equal(etc.etc_get_solution(plan).cpu().numpy(), e_p), rep
        assert etc.etc_keff(plan)["keff"] == e_k, rep
        assert np.array_equal(etc.etc_grad(plan).cpu().numpy(), e_g), rep
        torch.cuda.synchronize()
    plan.close()


def test_graph_batch_and_side_stream():
    """Graph replay on a caller's side stream and on a batch plan."""
    n = 20
    kaps = np.stack([lognormal((n, n, n), seed=90 + i, sigma=0.3 + 0.4 * i) for i in range(3)])
    ref = etc.solve_batch(dev(kaps), 1, rtol=1e-9)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = etc.solve_batch(dev(kaps), 1, rtol=1e-9, use_graph=True)
    torch.cuda.synchronize()
    assert out["iters"] == ref["iters"]
    assert out["keff"] == ref["keff"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_batch_with_persistent_column_kernels(precision):
    """Graph replay on a batch whose column length (64) has the persistent
    column kernels and whose instances converge at different passes: the
    plan keeps one captured graph per converged-instance state (persistent
    column kernels until an instance converges, gated ones after), so the
    replayed passes launch what the eager passes launch and give the same
    pass counts and K_eff bit for bit."""
    shape = (16, 64, 64)
    kaps = np.stack([np.exp(s * np.random.default_rng(300 + i).standard_normal(shape))
                     for i, s in enumerate([0.1, 0.8, 1.5])])
    rtol = 1e-10 if precision == "fp64" else 1e-6
    eager = etc.solve_batch(dev(kaps), 0, precision=precision, rtol=rtol)
    graph = etc.solve_batch(dev(kaps), 0, precision=precision, rtol=rtol, use_graph=True)
    assert len(set(eager["iters"])) > 1
    assert graph["status"] == eager["status"]
    assert graph["iters"] == eager["iters"]
    assert graph["keff"] == eager["keff"]


# --------------------------------------------------------------- ensembles
@pytest.mark.parametrize("concurrent", [True, False])
def test_ensemble_of_mixed_sizes_matches_oracle(concurrent):
    """solve_ensemble(mode="plans") buckets RVEs by shape into batch plans
    (split when a bucket exceeds the voxel cap), runs the plans one after
    another or at the same time on streams of their own, and returns results
    in input order; each K_eff equals the oracle's, gradients included."""
    edges = [12, 16, 12, 20, 16, 12]
    kaps_np = [rvegen.grf_lognormal(n, 1.0 + 0.2 * i, 4.0, 600 + i, dtype=np.float64) for i, n in enumerate(edges)]
    out = etc.solve_ensemble([dev(k) for k in kaps_np], 1, max_batch_voxels=2 * 12 ** 3, rtol=1e-11,
                             want_grad=True, concurrent=concurrent, mode="plans")
    # cap of two 12^3 RVEs: 12^3 x3 -> 2 plans, 16^3 x2 -> 2 plans, 20^3 -> 1 plan
    assert out["plans"] == 5
    for i, k in enumerate(kaps_np):
        ref = O.solve(k, 1, rtol=1e-13)
        assert out["status"][i] == "ok"
        assert abs(out["keff"][i] - ref["keff"]) <= 1e-9 * ref["keff"], i
        gref = O.decanonical(O.keff_gradient(ref["problem"], ref["pcg"].p), 1)
        g = out["grad"][i].cpu().numpy()
        assert g.shape == k.shape
        assert np.abs(g - gref).max() <= 1e-7 * np.abs(gref).max(), i


# ---------------------------------------------------------------- autotuner
def test_autotuned_plan_reaches_the_same_solution():
    """The setup-time autotuner only changes launch shapes: the solve reaches
    the oracle's K_eff, and a second plan of the same shape reuses the
    choice."""
    kap = lognormal((40, 72, 48), seed=61, sigma=1.0)
    ref = O.solve(kap, 0, rtol=1e-12)
    for precision, tol in (("fp64", 1e-9), ("mixed", 1e-5)):
        plan = etc.etc_setup(dev(kap), 0, rtol=1e-10 if precision == "fp64" else 1e-6, precision=precision,
                             autotune=True)
        info = etc.etc_launch_info(plan)
        assert info["tuned"] and 1 <= info["kchunk"] <= 40 and info["thomas_blocks"] >= 1
        assert info["thomas_shape"] in [(32, 8), (16, 16), (32, 16), (64, 8), (32, 32), (16, 32)]
        etc.etc_solve(plan)
        k = etc.etc_keff(plan)["keff"]
        plan.close()
        assert abs(k - ref["keff"]) <= tol * ref["keff"]
        again = etc.etc_setup(dev(kap), 0, precision=precision, autotune=True)
        assert etc.etc_launch_info(again) == info
        again.close()
    plain = etc.etc_setup(dev(kap), 0)
    assert not etc.etc_launch_info(plain)["tuned"]
    plain.close()
