"""Plain FP64 CPU oracle for TPFA effective thermal conductivity with the
DCT/Thomas-preconditioned conjugate gradient method (Ye, Fu and Chung,
arXiv 2404.02433).

TEST INFRASTRUCTURE.  This module exists to check the GPU library.  Only the
test-suite, the package smoke check and the benchmark's CPU-baseline leg may
import it; the product path never calls it.  It shares no code with the GPU
path (no kernels, tables, constants or helpers); both sides only consume the
same seeded conductivity arrays.

Everything is float64 NumPy, written to be read against the paper:

* canonical layout ``[k][a][b]``: the Dirichlet (load) axis ``k`` first, the two
  transverse axes after it in their original order;
* ``h`` holds the voxel edge per canonical axis (the paper's h^x, h^y, h^z with
  h = L/N); the scaled coefficients are kappa~ = kappa / h^2 (Section
  "Discretization scheme", scaling before eq:scaled bilinear forms).

Every public function is pinned by ``tests/test_oracle_pins.py`` against
facts the paper or mathematics fix (library transforms, dense solves, exact
laminate and homogeneous cases, bounds, the spectral lemma, the LP optimum,
Tables 1 and 2, finite differences); the layout helpers marked "helper"
only move axes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "canonical", "decanonical", "Problem", "make_problem",
    "apply_A", "apply_A_at", "rhs", "dense_A",
    "family_extrema", "kref_mid", "lemma_bounds",
    "dct2", "dct3", "cos_matrix", "neumann_eigenvalues",
    "thomas", "apply_Aref_inv", "apply_Aref_at", "dense_Aref",
    "PCGResult", "pcg", "keff", "solve",
    "keff_gradient",
]


# ---------------------------------------------------------------------------
# Layout
# ---------------------------------------------------------------------------

def canonical(kappa: np.ndarray, axis: int) -> np.ndarray:
    """Move the load axis to the front; the other two keep their order (helper)."""
    return np.ascontiguousarray(np.moveaxis(np.asarray(kappa, dtype=np.float64), axis, 0))


def decanonical(x: np.ndarray, axis: int) -> np.ndarray:
    """Inverse of :func:`canonical` (helper)."""
    return np.ascontiguousarray(np.moveaxis(x, 0, axis))


@dataclass
class Problem:
    """Canonical TPFA problem: kappa[k, a, b], voxel edges, Dirichlet data.

    ``kap`` is the isotropic conductivity, or the load-axis component of an
    orthotropic one when ``kap_a`` / ``kap_b`` (components along the two
    transverse axes) are given (Section "Model problem": K = diag(kappa^x,
    kappa^y, kappa^z) per voxel).  ``p_in`` / ``p_out`` are constants or
    per-face arrays (na, nb) sampled at the Dirichlet face centres; ``src`` is
    an optional volume source f sampled at cell centres."""
    kap: np.ndarray            # (nL, na, nb) float64, > 0
    h: tuple                   # voxel edge per canonical axis (hL, ha, hb)
    p_in: object = 1.0
    p_out: object = 0.0
    kap_a: np.ndarray = None
    kap_b: np.ndarray = None
    src: np.ndarray = None

    @property
    def shape(self):
        return self.kap.shape

    @property
    def kapA(self):
        return self.kap if self.kap_a is None else self.kap_a

    @property
    def kapB(self):
        return self.kap if self.kap_b is None else self.kap_b


def make_problem(kappa, axis: int = 0, p_in=1.0, p_out=0.0, L=None, components=None, source=None) -> Problem:
    """Canonicalise user-layout data.  ``L`` = domain lengths per user axis
    (default: cubic voxels of edge 1).  ``components`` = three arrays, the
    conductivity along user axes 0, 1, 2 (orthotropic K; ``kappa`` is then
    ignored).  ``p_in`` / ``p_out`` may be arrays over the two transverse user
    axes (in their user order); ``source`` a user-layout array."""
    order = [axis] + [d for d in range(3) if d != axis]
    if components is not None:
        comps = [canonical(c, axis) for c in components]
        kap, kap_a, kap_b = comps[order[0]], comps[order[1]], comps[order[2]]
        n_user = np.asarray(components[0]).shape
    else:
        kap, kap_a, kap_b = canonical(kappa, axis), None, None
        n_user = np.asarray(kappa).shape
    if L is None:
        h_user = (1.0, 1.0, 1.0)
    else:
        h_user = tuple(float(L[d]) / n_user[d] for d in range(3))
    face = lambda v: float(v) if np.isscalar(v) else np.asarray(v, dtype=np.float64)
    src = None if source is None else canonical(source, axis)
    return Problem(kap, tuple(h_user[d] for d in order), face(p_in), face(p_out), kap_a, kap_b, src)


# ---------------------------------------------------------------------------
# TPFA operator (Section "Discretization scheme")
# ---------------------------------------------------------------------------

def _harmonic(k1, k2):
    """Internal-face conductivity: the harmonic mean 2 / (1/k1 + 1/k2) that
    the trapezoidal mass lumping produces for a face shared by two cells."""
    return 2.0 / (1.0 / k1 + 1.0 / k2)


def _faces(pb: Problem):
    """Scaled face transmissibilities of eq:scaled bilinear forms.

    Returns (TL, Ta, Tb, Tin, Tout): internal faces normal to each canonical
    axis (harmonic means of kappa~ of the two cells), and the Dirichlet-face
    coefficients 2 kappa~ of the first and last load layers (a^in, a^out).
    """
    hL, ha, hb = pb.h
    kL, ka, kb = pb.kap / hL ** 2, pb.kapA / ha ** 2, pb.kapB / hb ** 2
    TL = _harmonic(kL[1:], kL[:-1])
    Ta = _harmonic(ka[:, 1:], ka[:, :-1])
    Tb = _harmonic(kb[:, :, 1:], kb[:, :, :-1])
    return TL, Ta, Tb, 2.0 * kL[0], 2.0 * kL[-1]


def apply_A(pb: Problem, p: np.ndarray) -> np.ndarray:
    """Matrix of the bilinear form a = a* + a^in + a^out (eq:scaled bilinear forms)
    applied to a cell vector: sum over faces of kappa_F times the face jump,
    plus 2 kappa~ p on the two Dirichlet layers."""
    TL, Ta, Tb, Tin, Tout = _faces(pb)
    q = np.zeros_like(p)
    f = TL * (p[1:] - p[:-1])
    q[1:] += f
    q[:-1] -= f
    f = Ta * (p[:, 1:] - p[:, :-1])
    q[:, 1:] += f
    q[:, :-1] -= f
    f = Tb * (p[:, :, 1:] - p[:, :, :-1])
    q[:, :, 1:] += f
    q[:, :, :-1] -= f
    q[0] += Tin * p[0]
    q[-1] += Tout * p[-1]
    return q


def apply_A_at(pb: Problem, p: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """(A p) at the canonical voxels ``idx`` (rows of (k, a, b)), one voxel at
    a time from the same definition as apply_A: for each of the six faces,
    the harmonic mean of kappa~ of the two cells times (p_c - p_n) when the
    neighbour exists, and 2 kappa~ p_c for a face on a Dirichlet layer.  For
    sampled checks on grids too large for whole-array evaluation."""
    hL, ha, hb = pb.h
    sc = (hL ** -2, ha ** -2, hb ** -2)
    comps = (pb.kap, pb.kapA, pb.kapB)
    shape = pb.shape
    out = np.empty(len(idx))
    for n, (k, a, b) in enumerate(np.asarray(idx, dtype=np.int64)):
        c = (k, a, b)
        pc = p[c]
        acc = 0.0
        for d in range(3):
            kc = comps[d][c] * sc[d]
            for step in (-1, 1):
                nb_ = list(c)
                nb_[d] += step
                if 0 <= nb_[d] < shape[d]:
                    kn = comps[d][tuple(nb_)] * sc[d]
                    acc += _harmonic(kc, kn) * (pc - p[tuple(nb_)])
                elif d == 0:
                    acc += 2.0 * kc * pc
        out[n] = acc
    return out


def rhs(pb: Problem) -> np.ndarray:
    """Right-hand side from the Dirichlet data.  Substituting the discrete flux
    eq:flux (with p~_F = -p_in on Gamma_in, p_out on Gamma_out and zero ghost
    values) into the cell balance puts 2 kappa~ p_in on the first load layer
    and 2 kappa~ p_out on the last one; every other entry is zero.  A volume
    source f adds f at each cell (the balance divided by the cell volume)."""
    _, _, _, Tin, Tout = _faces(pb)
    b = np.zeros(pb.shape)
    b[0] += Tin * pb.p_in
    b[-1] += Tout * pb.p_out
    if pb.src is not None:
        b += pb.src
    return b


def dense_A(pb: Problem) -> np.ndarray:
    """Assemble A densely face by face from the bilinear form, with explicit
    loops (small grids only)."""
    nL, na, nb = pb.shape
    TL, Ta, Tb, Tin, Tout = _faces(pb)
    idx = lambda k, a, b: (k * na + a) * nb + b
    A = np.zeros((nL * na * nb,) * 2)

    def face(c, n, t):
        A[c, c] += t
        A[n, n] += t
        A[c, n] -= t
        A[n, c] -= t

    for k in range(nL):
        for a in range(na):
            for b in range(nb):
                c = idx(k, a, b)
                if k > 0:
                    face(c, idx(k - 1, a, b), TL[k - 1, a, b])
                if a > 0:
                    face(c, idx(k, a - 1, b), Ta[k, a - 1, b])
                if b > 0:
                    face(c, idx(k, a, b - 1), Tb[k, a, b - 1])
    for a in range(na):
        for b in range(nb):
            A[idx(0, a, b), idx(0, a, b)] += Tin[a, b]
            A[idx(nL - 1, a, b), idx(nL - 1, a, b)] += Tout[a, b]
    return A


# ---------------------------------------------------------------------------
# Reference medium (eq:refer bilinear forms, eq:parameters for linear
# programming, eq:linear programming, alg:refer parameters)
# ---------------------------------------------------------------------------

FAMILIES = ("L", "a", "b", "in", "out")


def family_extrema(pb: Problem) -> dict:
    """Min and max of each coefficient family of eq:parameters for linear
    programming: internal harmonic-mean faces normal to each axis, and the
    scaled load-axis conductivity of the first (in) and last (out) layers.
    An empty family (an axis of length 1) is reported as None."""
    TL, Ta, Tb, Tin, Tout = _faces(pb)
    out = {}
    for name, arr in (("L", TL), ("a", Ta), ("b", Tb), ("in", 0.5 * Tin), ("out", 0.5 * Tout)):
        out[name] = None if arr.size == 0 else (float(arr.min()), float(arr.max()))
    return out


def kref_mid(pb: Problem) -> dict:
    """Reference parameters as the geometric midpoint sqrt(min * max) of each
    family.  This is one optimal point of the linear programme in
    eq:linear programming: its objective max_d ln(max_d/min_d) is the LP's
    optimal value (the programme's optimum is not unique; this reading is the
    symmetric one).  Empty families get 1 (they never enter the solve)."""
    ext = family_extrema(pb)
    return {f: (1.0 if ext[f] is None else math.sqrt(ext[f][0] * ext[f][1])) for f in FAMILIES}


def lemma_bounds(pb: Problem, kref: dict):
    """Lambda' and Lambda'' of lem:cond: the smallest and largest ratio of a
    family extremum to its reference value (the out-layer ratio uses the out
    reference)."""
    ext = family_extrema(pb)
    lo = min(ext[f][0] / kref[f] for f in FAMILIES if ext[f] is not None)
    hi = max(ext[f][1] / kref[f] for f in FAMILIES if ext[f] is not None)
    return lo, hi


# ---------------------------------------------------------------------------
# 1D DCT pair (eq:forward DCT, eq:backword DCT) and the Neumann eigenpairs
# ---------------------------------------------------------------------------

def cos_matrix(N: int) -> np.ndarray:
    """C[k', i] = cos(pi (2i+1) k' / (2N)), the kernel of eq:forward DCT."""
    i = np.arange(N)
    return np.cos(np.pi * np.outer(np.arange(N), 2 * i + 1) / (2 * N))


def dct2(x: np.ndarray, axis: int) -> np.ndarray:
    """Forward DCT (scale 1) along ``axis``, by its O(N^2) definition."""
    N = x.shape[axis]
    C = cos_matrix(N)
    return np.moveaxis(np.tensordot(C, np.moveaxis(x, axis, 0), axes=(1, 0)), 0, axis)


def dct3(X: np.ndarray, axis: int) -> np.ndarray:
    """Backward DCT: (2/N) sum_k' alpha_k' X_k' cos(...), alpha_0 = 1/2, by its
    O(N^2) definition."""
    N = X.shape[axis]
    C = cos_matrix(N)
    alpha = np.ones(N)
    alpha[0] = 0.5
    W = (2.0 / N) * (C.T * alpha[None, :])
    return np.moveaxis(np.tensordot(W, np.moveaxis(X, axis, 0), axes=(1, 0)), 0, axis)


def neumann_eigenvalues(N: int) -> np.ndarray:
    """lambda_k = 2 (1 - cos(k pi / N)) of the 1D Neumann matrix tridiag(-1, 2, -1)
    with unit corners; its eigenvectors are the rows of :func:`cos_matrix`."""
    return 2.0 * (1.0 - np.cos(np.arange(N) * np.pi / N))


# ---------------------------------------------------------------------------
# Preconditioner solve (alg:solve ref)
# ---------------------------------------------------------------------------

def thomas(lower, diag, upper, d):
    """Tridiagonal solve without pivoting, batched over trailing dimensions.

    ``diag`` and ``d`` have shape (n, ...); ``lower[k]`` couples row k to row
    k-1 (lower[0] unused), ``upper[k]`` couples row k to row k+1 (upper[-1]
    unused).  Forward elimination then back substitution."""
    n = d.shape[0]
    cp = np.empty_like(d)
    dp = np.empty_like(d)
    cp[0] = upper[0] / diag[0]
    dp[0] = d[0] / diag[0]
    for k in range(1, n):
        den = diag[k] - lower[k] * cp[k - 1]
        cp[k] = upper[k] / den if k < n - 1 else 0.0
        dp[k] = (d[k] - lower[k] * dp[k - 1]) / den
    x = np.empty_like(d)
    x[-1] = dp[-1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def _T_diagonals(shape, kref):
    """Diagonals of the tridiagonal matrices T_{a',b'} (Section "Preconditioner
    system solver"): shift (lambda_a kappa_ref^a + lambda_b kappa_ref^b) plus
    kappa_ref^L tridiag(-1, 2, -1) whose first and last diagonal entries are
    kappa_ref^L + 2 kappa_ref^in and kappa_ref^L + 2 kappa_ref^out."""
    nL, na, nb = shape
    s = (neumann_eigenvalues(na)[:, None] * kref["a"] + neumann_eigenvalues(nb)[None, :] * kref["b"])
    kz = kref["L"]
    diag = np.empty((nL, na, nb))
    diag[:] = s + 2.0 * kz
    diag[0] = s + kz + 2.0 * kref["in"]
    diag[-1] = s + kz + 2.0 * kref["out"]
    off = np.full((nL, na, nb), -kz)
    return off, diag, off


def apply_Aref_inv(r: np.ndarray, kref: dict) -> np.ndarray:
    """z = A_ref^{-1} r by alg:solve ref: forward 2D DCT of every load plane,
    one tridiagonal solve per transverse mode (a', b'), backward 2D DCT."""
    rh = dct2(dct2(r, 1), 2)
    lo, dg, up = _T_diagonals(r.shape, kref)
    zh = thomas(lo, dg, up, rh)
    return dct3(dct3(zh, 2), 1)


def apply_Aref_at(z: np.ndarray, kref: dict, idx: np.ndarray) -> np.ndarray:
    """(A_ref z) at the canonical voxels ``idx``, one voxel at a time from
    eq:refer bilinear forms: constant coefficients kappa_ref^L, ^a, ^b on the
    internal faces normal to each axis, 2 kappa_ref^in and 2 kappa_ref^out on
    the two Dirichlet layers, nothing on the Neumann faces."""
    coef = (kref["L"], kref["a"], kref["b"])
    shape = z.shape
    out = np.empty(len(idx))
    for n, (k, a, b) in enumerate(np.asarray(idx, dtype=np.int64)):
        c = (k, a, b)
        zc = z[c]
        acc = 0.0
        for d in range(3):
            for step in (-1, 1):
                nb_ = list(c)
                nb_[d] += step
                if 0 <= nb_[d] < shape[d]:
                    acc += coef[d] * (zc - z[tuple(nb_)])
        if k == 0:
            acc += 2.0 * kref["in"] * zc
        if k == shape[0] - 1:
            acc += 2.0 * kref["out"] * zc
        out[n] = acc
    return out


def dense_Aref(shape, kref: dict) -> np.ndarray:
    """A_ref assembled from eq:refer bilinear forms as a sum of Kronecker
    products of 1D matrices (small grids only)."""
    nL, na, nb = shape

    def neumann(N):
        M = np.zeros((N, N))
        for i in range(N - 1):
            M[i, i] += 1
            M[i + 1, i + 1] += 1
            M[i, i + 1] -= 1
            M[i + 1, i] -= 1
        return M

    IL, Ia, Ib = np.eye(nL), np.eye(na), np.eye(nb)
    Dz = np.zeros((nL, nL))
    Dz[0, 0] += 2 * kref["in"]
    Dz[-1, -1] += 2 * kref["out"]
    return (np.kron(kref["L"] * neumann(nL) + Dz, np.kron(Ia, Ib))
            + kref["a"] * np.kron(IL, np.kron(neumann(na), Ib))
            + kref["b"] * np.kron(IL, np.kron(Ia, neumann(nb))))


# ---------------------------------------------------------------------------
# PCG (alg:pcg) with the exit test eq:exit
# ---------------------------------------------------------------------------

@dataclass
class PCGResult:
    p: np.ndarray
    iters: int
    converged: bool
    relres: float
    history: list = field(default_factory=list)
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)
    status: str = "ok"


def pcg(pb: Problem, rtol: float = 1e-6, max_iter: int = 1000, kref: dict | None = None,
        precond: bool = True, p0: np.ndarray | None = None) -> PCGResult:
    """alg:pcg with p0 = 0 by default.  The exit test eq:exit (||r|| / ||b|| <=
    rtol, r the recursively updated residual) is taken at the top of every
    pass; ``iters`` counts the passes, i.e. the products A w."""
    if kref is None:
        kref = kref_mid(pb)
    b = rhs(pb)
    bnorm = float(np.linalg.norm(b))
    p = np.zeros(pb.shape) if p0 is None else np.array(p0, dtype=np.float64)
    r = b - apply_A(pb, p)
    M = (lambda v: apply_Aref_inv(v, kref)) if precond else (lambda v: v.copy())
    z = M(r)
    w = z.copy()
    rho = float(np.vdot(r, z))
    res = PCGResult(p, 0, False, float(np.linalg.norm(r)) / bnorm)
    res.history.append(res.relres)
    it = 0
    while True:
        relres = float(np.linalg.norm(r)) / bnorm
        if relres <= rtol:
            res.converged = True
            break
        if it >= max_iter:
            res.status = "not_converged"
            break
        q = apply_A(pb, w)
        wq = float(np.vdot(q, w))
        if not (wq > 0.0) or not math.isfinite(wq):
            res.status = "breakdown"
            break
        alpha = rho / wq
        p += alpha * w
        r -= alpha * q
        it += 1
        res.alphas.append(alpha)
        res.history.append(float(np.linalg.norm(r)) / bnorm)
        z = M(r)
        rho_new = float(np.vdot(r, z))
        beta = rho_new / rho
        res.betas.append(beta)
        w = z + beta * w
        rho = rho_new
    res.p, res.iters, res.relres = p, it, float(np.linalg.norm(r)) / bnorm
    return res


# ---------------------------------------------------------------------------
# Effective conductivity (eq:effective formula dis with eq:flux)
# ---------------------------------------------------------------------------

def keff(pb: Problem, p: np.ndarray) -> dict:
    """Effective conductivity along the load axis.

    ``out``: eq:effective formula dis, L^z times the summed outflow-face flux
    over N^x N^y (p_in - p_out); by eq:flux the flux through an outflow face is
    2 kappa (p_last - p_out) / h^z, and L^z / h^z = N^z.
    ``in``: the same with the inflow faces (flux 2 kappa (p_in - p_first)/h^z);
    equal to ``out`` at the exact solution because the two boundary flux
    integrals cancel (Section "Model problem").
    ``energy``: N^z h^z^2 E / (N^x N^y dp^2) with E the discrete dissipation
    sum_F kappa_F (jump)^2 including the Dirichlet faces; equal to ``out`` at
    the exact solution (E = Q dp)."""
    nL, na, nb = pb.shape
    hL = pb.h[0]
    dp = pb.p_in - pb.p_out
    k_out = nL * float(np.sum(2.0 * pb.kap[-1] * (p[-1] - pb.p_out))) / (na * nb * dp)
    k_in = nL * float(np.sum(2.0 * pb.kap[0] * (pb.p_in - p[0]))) / (na * nb * dp)
    TL, Ta, Tb, Tin, Tout = _faces(pb)
    E = (float(np.sum(TL * (p[1:] - p[:-1]) ** 2)) + float(np.sum(Ta * (p[:, 1:] - p[:, :-1]) ** 2))
         + float(np.sum(Tb * (p[:, :, 1:] - p[:, :, :-1]) ** 2))
         + float(np.sum(Tin * (p[0] - pb.p_in) ** 2)) + float(np.sum(Tout * (p[-1] - pb.p_out) ** 2)))
    k_en = nL * hL ** 2 * E / (na * nb * dp * dp)
    return {"out": k_out, "in": k_in, "energy": k_en}


def solve(kappa, axis: int = 0, p_in: float = 1.0, p_out: float = 0.0, rtol: float = 1e-6,
          max_iter: int = 1000, L=None, kref: dict | None = None) -> dict:
    """Whole routine of the discretisation section: solve A p = b by PCG,
    reconstruct the boundary flux, return K_eff (and diagnostics)."""
    pb = make_problem(kappa, axis, p_in, p_out, L)
    if kref is None:
        kref = kref_mid(pb)
    res = pcg(pb, rtol=rtol, max_iter=max_iter, kref=kref)
    k = keff(pb, res.p)
    return {"keff": k["out"], "k_in": k["in"], "k_energy": k["energy"], "iters": res.iters,
            "relres": res.relres, "converged": res.converged, "kref": kref, "pcg": res, "problem": pb}


# ---------------------------------------------------------------------------
# Gradient of K_eff with respect to every voxel conductivity
# ---------------------------------------------------------------------------

def keff_gradient(pb: Problem, p: np.ndarray) -> np.ndarray:
    """dK_out/dkappa for every voxel (canonical layout), from the energy form.

    At the exact solution K_out = K_energy = c E(p), E the dissipation in
    :func:`keff`, and E is stationary in p (p minimises E under the Dirichlet
    data), so dK/dkappa_v = c dE/dkappa_v at fixed p: a sum over the faces of
    voxel v of d(kappa_F)/d(kappa_v) times the squared face jump.  For a
    harmonic-mean face 2 k1 k2/(k1 + k2), d/dk1 = 2 k2^2 / (k1 + k2)^2; for a
    Dirichlet face 2 kappa~, the derivative is 2 / h^2."""
    nL, na, nb = pb.shape
    hL, ha, hb = pb.h
    dp = pb.p_in - pb.p_out
    c = nL * hL ** 2 / (na * nb * dp * dp)
    k = pb.kap
    g = np.zeros_like(k)

    def face_grad(k1, k2, jump2, h2, sl1, sl2):
        # kappa_F = 2 (k1/h2)(k2/h2) / ((k1 + k2)/h2) = 2 k1 k2 / ((k1 + k2) h2)
        s = (k1 + k2) ** 2
        g[sl1] += 2.0 * k2 * k2 / s / h2 * jump2
        g[sl2] += 2.0 * k1 * k1 / s / h2 * jump2

    face_grad(k[1:], k[:-1], (p[1:] - p[:-1]) ** 2, hL ** 2, np.s_[1:], np.s_[:-1])
    face_grad(k[:, 1:], k[:, :-1], (p[:, 1:] - p[:, :-1]) ** 2, ha ** 2, np.s_[:, 1:], np.s_[:, :-1])
    face_grad(k[:, :, 1:], k[:, :, :-1], (p[:, :, 1:] - p[:, :, :-1]) ** 2, hb ** 2,
              np.s_[:, :, 1:], np.s_[:, :, :-1])
    g[0] += 2.0 / hL ** 2 * (p[0] - pb.p_in) ** 2
    g[-1] += 2.0 / hL ** 2 * (p[-1] - pb.p_out) ** 2
    return c * g
