"""Pins of the oracle's projection step (Section 3.3: the right-hand side
alpha D u of the pressure equation and the velocity update u -= beta G psi,
on the staggered layout of Section 3).

Each pin fixes the oracle by something other than its own formula:
  * flux conservation: the divergence sums to zero over the box (periodic
    directions wrap, walls carry no flux);
  * a single unit flux on one face gives +1/h in the cell it leaves and
    -1/h in the cell it enters (face convention and sign), or only the
    first when the face is a wall;
  * D G = L: the divergence of the face gradient is the 7-point Laplacian
    (pinned independently by eigenmodes and dense LU in
    test_oracle_pins.py);
  * the input generator's own divergence (written separately) agrees;
  * after a solve, the corrected velocity is divergence-free to rounding;
  * a uniform psi leaves the velocity unchanged.
"""
import numpy as np
import pytest

from paper_2204_08834_amd import inputs

NEU, PER = 1, 0


def _vel(shape, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1, 1, shape) for _ in range(3)]


@pytest.mark.parametrize("bc", [NEU, PER])
def test_divergence_conserves_flux(orc, bc):
    u, v, w = _vel((6, 5, 7), 1)
    f = orc.divergence(u, v, w, 0.1, 0.2, 0.3, bc)
    assert abs(f.sum()) <= 1e-12 * np.abs(f).sum()


@pytest.mark.parametrize("bc", [NEU, PER])
def test_unit_face_flux(orc, bc):
    nz, ny, nx = 4, 3, 5
    dx, dy, dz = 0.5, 0.25, 0.125
    z = np.zeros((nz, ny, nx))
    # east face of cell (k=1, j=2, i=4): leaves cell i=4, enters i=0 (wrap)
    u = z.copy()
    u[1, 2, 4] = 1.0
    f = orc.divergence(u, z, z, dx, dy, dz, bc)
    exp = np.zeros_like(z)
    exp[1, 2, 4] = 1 / dx
    exp[1, 2, 0] = -1 / dx
    assert np.array_equal(f, exp)
    # north face of cell (k=2, j=1, i=3): enters j=2
    v = z.copy()
    v[2, 1, 3] = 1.0
    f = orc.divergence(z, v, z, dx, dy, dz, bc)
    exp = np.zeros_like(z)
    exp[2, 1, 3] = 1 / dy
    exp[2, 2, 3] = -1 / dy
    assert np.array_equal(f, exp)
    # top face of the last cell: the wall (no flux), or wraps to k = 0
    w = z.copy()
    w[nz - 1, 0, 2] = 1.0
    f = orc.divergence(z, z, w, dx, dy, dz, bc)
    exp = np.zeros_like(z)
    if bc == PER:
        exp[nz - 1, 0, 2] = 1 / dz
        exp[0, 0, 2] = -1 / dz
    assert np.array_equal(f, exp)
    # an interior top face
    w = z.copy()
    w[1, 0, 2] = 1.0
    f = orc.divergence(z, z, w, dx, dy, dz, bc)
    exp = np.zeros_like(z)
    exp[1, 0, 2] = 1 / dz
    exp[2, 0, 2] = -1 / dz
    assert np.array_equal(f, exp)


@pytest.mark.parametrize("bc", [NEU, PER])
def test_divergence_of_gradient_is_laplacian(orc, bc):
    rng = np.random.default_rng(3)
    psi = rng.uniform(-1, 1, (6, 7, 8))
    sp = (0.3, 0.2, 0.1)
    z = np.zeros_like(psi)
    gu, gv, gw = orc.correct(z, z, z, psi, *sp, bc, beta=-1.0)  # +G psi
    lap = orc.laplacian(psi, *sp, bc)
    dg = orc.divergence(gu, gv, gw, *sp, bc)
    assert np.max(np.abs(dg - lap)) <= 1e-12 * np.max(np.abs(lap))


@pytest.mark.parametrize("bc", [NEU, PER])
def test_matches_generator_divergence(orc, bc):
    u, v, w = _vel((5, 6, 4), 4)
    if bc == NEU:
        w[-1] = 0.0
    sp = (0.25, 0.5, 0.125)
    a = orc.divergence(u, v, w, *sp, bc)
    b = inputs.divergence(u, v, w, *sp, bc)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("bc", [NEU, PER])
def test_projection_is_divergence_free(orc, bc):
    u, v, w = _vel((8, 12, 16), 5)
    sp = (1 / 16, 1 / 12, 1 / 8)
    alpha = 7.0
    psi, (u2, v2, w2) = orc.project(u, v, w, *sp, bc, alpha=alpha, beta=1 / alpha)
    d0 = orc.divergence(u, v, w, *sp, bc)
    d1 = orc.divergence(u2, v2, w2, *sp, bc)
    assert np.max(np.abs(d1)) <= 1e-12 * np.max(np.abs(d0))
    if bc == NEU:
        assert np.array_equal(w2[-1], w[-1])  # the wall face is not touched


def test_uniform_psi_leaves_velocity(orc):
    u, v, w = _vel((3, 4, 5), 6)
    psi = np.full((3, 4, 5), 2.5)
    u2, v2, w2 = orc.correct(u, v, w, psi, 0.1, 0.2, 0.3, NEU, beta=3.0)
    assert np.array_equal(u2, u) and np.array_equal(v2, v) and np.array_equal(w2, w)


# --------------------------------------------------------------------------
# solid walls along x and y as well
# --------------------------------------------------------------------------
WALL_SETS = [(NEU, NEU, NEU), (NEU, PER, NEU), (PER, NEU, PER), (NEU, NEU, PER)]


@pytest.mark.parametrize("bcs", WALL_SETS)
def test_walls_divergence_conserves_flux(orc, bcs):
    u, v, w = _vel((5, 6, 7), 11)
    f = orc.divergence(u, v, w, 0.1, 0.2, 0.3, bcs[2], bc_x=bcs[0], bc_y=bcs[1])
    assert abs(f.sum()) <= 1e-12 * np.abs(f).sum()


def test_walls_unit_face_flux(orc):
    """With walls along x and y the last faces carry nothing; an interior
    face moves +1/h to -1/h as before."""
    nz, ny, nx = 3, 4, 5
    dx, dy, dz = 0.5, 0.25, 0.125
    z = np.zeros((nz, ny, nx))
    for axis, (i, j, k) in (("u", (nx - 1, 2, 1)), ("v", (3, ny - 1, 2))):
        a = z.copy()
        a[k, j, i] = 1.0
        args = (a, z, z) if axis == "u" else (z, a, z)
        f = orc.divergence(*args, dx, dy, dz, NEU, bc_x=NEU, bc_y=NEU)
        assert np.array_equal(f, z), axis  # the wall face is not read
    a = z.copy()
    a[1, 2, 1] = 1.0
    f = orc.divergence(a, z, z, dx, dy, dz, NEU, bc_x=NEU, bc_y=NEU)
    exp = z.copy()
    exp[1, 2, 1] = 1 / dx
    exp[1, 2, 2] = -1 / dx
    assert np.array_equal(f, exp)


@pytest.mark.parametrize("bcs", WALL_SETS)
def test_walls_divergence_of_gradient_is_laplacian(orc, bcs):
    rng = np.random.default_rng(13)
    psi = rng.uniform(-1, 1, (6, 7, 8))
    sp = (0.3, 0.2, 0.1)
    z = np.zeros_like(psi)
    gu, gv, gw = orc.correct(z, z, z, psi, *sp, bcs[2], beta=-1.0, bc_x=bcs[0], bc_y=bcs[1])
    lap = orc.laplacian(psi, *sp, bcs[2], bc_x=bcs[0], bc_y=bcs[1])
    dg = orc.divergence(gu, gv, gw, *sp, bcs[2], bc_x=bcs[0], bc_y=bcs[1])
    assert np.max(np.abs(dg - lap)) <= 1e-12 * np.max(np.abs(lap))


@pytest.mark.parametrize("bcs", WALL_SETS)
def test_walls_projection_is_divergence_free(orc, bcs):
    u, v, w = _vel((8, 12, 16), 15)
    sp = (1 / 16, 1 / 12, 1 / 8)
    psi, (u2, v2, w2) = orc.project(u, v, w, *sp, bcs[2], alpha=4.0, beta=0.25, bc_x=bcs[0],
                                    bc_y=bcs[1])
    d0 = orc.divergence(u, v, w, *sp, bcs[2], bc_x=bcs[0], bc_y=bcs[1])
    d1 = orc.divergence(u2, v2, w2, *sp, bcs[2], bc_x=bcs[0], bc_y=bcs[1])
    assert np.max(np.abs(d1)) <= 1e-12 * np.max(np.abs(d0))
    if bcs[0] == NEU:
        assert np.array_equal(u2[:, :, -1], u[:, :, -1])
    if bcs[1] == NEU:
        assert np.array_equal(v2[:, -1, :], v[:, -1, :])
