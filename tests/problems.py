"""Test inputs built from closed forms (no solver arithmetic)."""

import numpy as np


def smooth_problem(n):
    """The smooth orthotropic manufactured solution of tab:smooth on the unit
    cube, sampled at cell centres (conductivity components along x, y, z and
    the source f = -div(K grad p)) and at the centres of the Dirichlet faces
    z = 0 and z = 1.  Returns (components, source, p_in_face, p_out_face,
    exact), all in the [x][y][z] user layout with z the load axis."""
    c = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    kx, ky, kz = np.cos(np.pi * Y) + 2, 2 * np.exp(Z), 3 * np.cos(np.pi * X) + 4
    exact = np.cos(np.pi * X) * np.cos(np.pi * Y) * np.exp(Z)
    # each component is constant along its own axis, so
    # -div(K grad p) = p (pi^2 (kx + ky) - kz) with the exact p above
    f = exact * (np.pi ** 2 * (np.cos(np.pi * Y) + 2 + 2 * np.exp(Z)) - 3 * np.cos(np.pi * X) - 4)
    face = np.cos(np.pi * c)[:, None] * np.cos(np.pi * c)[None, :]
    return (kx, ky, kz), f, face * 1.0, face * np.e, exact
