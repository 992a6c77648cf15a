"""Pins of the oracle's z-stretched solve (walls in z, cells of thickness
h[k]): the conservative reading of the second-order stencil of Section 3 on
cells of different thickness, with the elimination along z of Section 3.3.1.

Every pin is independent of the oracle's code: the operator is assembled
cell by cell from face fluxes in numpy and solved densely (LAPACK), with the
volume-weighted gauge; the oracle's Laplacian and residual are compared with
that matrix; equal thicknesses reduce to the uniform oracle; the fluxes
telescope (sum h L p = 0 with no Dirichlet wall); and planted mistakes (the
face distance taken as one cell's thickness, an unweighted mean) are caught.
"""
import itertools

import numpy as np
import pytest

PER, NEU, DIR = 0, 1, 2


def thicknesses(nz, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.3, 1.7, nz) / nz


def ghost_coeffs(n, i, d, bc):
    """(neighbour index, factor) of the neighbour at offset d of cell i of n:
    periodic wrap, mirrored (Neumann) or negated (Dirichlet) wall cell."""
    j = i + d
    if 0 <= j < n:
        return j, 1.0
    if bc == PER:
        return j % n, 1.0
    return i, (1.0 if bc == NEU else -1.0)


def assemble(nx, ny, nz, dx, dy, h, bcs):
    """The operator as an (N, N) matrix, row by row from its definition:
    x and y three-point second differences with the ghost rules, z as the
    difference of the face fluxes over the cell thickness (flux through an
    interior face: value difference over the centre distance (h_k+h_k+1)/2;
    Neumann wall: none; Dirichlet wall: (0 - p) over h/2)."""
    N = nx * ny * nz
    A = np.zeros((N, N))
    idx = lambda k, j, i: (k * ny + j) * nx + i
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        r = idx(k, j, i)
        for d in (-1, 1):
            ii, fx = ghost_coeffs(nx, i, d, bcs[0])
            A[r, idx(k, j, ii)] += fx / dx ** 2
            jj, fy = ghost_coeffs(ny, j, d, bcs[1])
            A[r, idx(k, jj, i)] += fy / dy ** 2
        A[r, r] -= 2.0 / dx ** 2 + 2.0 / dy ** 2
        # z: fluxes through the top (k+1/2) and bottom (k-1/2) faces
        for kn in (k + 1, k - 1):
            if 0 <= kn < nz:
                g = 1.0 / (0.5 * (h[k] + h[kn]))
                A[r, idx(kn, j, i)] += g / h[k]
                A[r, r] -= g / h[k]
            elif bcs[2] == DIR:
                A[r, r] -= (1.0 / (0.5 * h[k])) / h[k]
    return A


def dense_solve(f, dx, dy, h, bcs):
    nz, ny, nx = f.shape
    A = assemble(nx, ny, nz, dx, dy, h, bcs)
    b = f.ravel()
    if DIR in bcs:
        return np.linalg.solve(A, b).reshape(f.shape), 0.0
    w = np.repeat(h, nx * ny)
    mean = (w @ b) / w.sum()
    N = b.size
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = A
    M[:N, N] = 1.0
    M[N, :N] = w
    sol = np.linalg.solve(M, np.concatenate([b - mean, [0.0]]))
    return sol[:N].reshape(f.shape), mean


GRIDS = [(4, 3, 5), (6, 4, 4), (1, 1, 7), (2, 5, 3), (4, 4, 1)]
BCS = [(x, y, z) for x in (PER, NEU, DIR) for y in (PER, NEU, DIR) for z in (NEU, DIR)]


@pytest.mark.parametrize("bcs", BCS, ids=["".join("PND"[b] for b in c) for c in BCS])
def test_stretched_solve_matches_dense(orc, bcs):
    for g, (nx, ny, nz) in enumerate(GRIDS):
        h = thicknesses(nz, 10 + g)
        dx, dy = 0.7 / nx, 1.3 / ny
        f = np.random.default_rng(20 + g).uniform(-1, 1, (nz, ny, nx))
        ref, mean = dense_solve(f, dx, dy, h, bcs)
        p, info = orc.solve(f, dx, dy, None, bcs[2], bc_x=bcs[0], bc_y=bcs[1], dz_cells=h,
                            return_info=True)
        err = np.linalg.norm(p - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, (bcs, (nx, ny, nz), err)
        assert abs(info["rhs_mean"] - mean) <= 1e-14
        if DIR not in bcs:  # volume-weighted gauge
            w = np.repeat(h, nx * ny).reshape(nz, ny, nx)
            assert abs((w * p).sum()) <= 1e-13 * np.abs(p).max() * w.sum()


@pytest.mark.parametrize("bcs", [(PER, PER, NEU), (NEU, DIR, NEU), (PER, NEU, DIR),
                                 (DIR, DIR, DIR)])
def test_stretched_laplacian_and_residual(orc, bcs):
    nx, ny, nz = 6, 4, 5
    h = thicknesses(nz, 3)
    dx, dy = 0.5, 0.25
    rng = np.random.default_rng(4)
    p = rng.uniform(-1, 1, (nz, ny, nx))
    f = rng.uniform(-1, 1, (nz, ny, nx))
    A = assemble(nx, ny, nz, dx, dy, h, bcs)
    lp = (A @ p.ravel()).reshape(p.shape)
    out = orc.laplacian(p, dx, dy, None, bcs[2], bc_x=bcs[0], bc_y=bcs[1], dz_cells=h)
    assert np.max(np.abs(out - lp)) <= 1e-13 * np.max(np.abs(lp))
    w = np.repeat(h, nx * ny).reshape(nz, ny, nx)
    fb = f - ((w * f).sum() / w.sum() if DIR not in bcs else 0.0)
    r = fb - lp
    l2, li = orc.residual(f, p, dx, dy, None, bcs[2], bc_x=bcs[0], bc_y=bcs[1], dz_cells=h)
    assert abs(l2 - np.linalg.norm(r) / np.linalg.norm(fb)) <= 1e-14 * l2
    assert abs(li - np.abs(r).max() / np.abs(fb).max()) <= 1e-14 * li


@pytest.mark.parametrize("bcs", [(PER, PER, NEU), (NEU, PER, DIR), (DIR, NEU, NEU)])
def test_equal_thicknesses_reduce_to_uniform(orc, bcs):
    nx, ny, nz = 8, 6, 10
    dz = 0.037
    f = np.random.default_rng(5).uniform(-1, 1, (nz, ny, nx))
    p_u = orc.solve(f, 0.1, 0.2, dz, bcs[2], bc_x=bcs[0], bc_y=bcs[1])
    p_s = orc.solve(f, 0.1, 0.2, None, bcs[2], bc_x=bcs[0], bc_y=bcs[1],
                    dz_cells=np.full(nz, dz))
    assert np.linalg.norm(p_s - p_u) <= 1e-13 * np.linalg.norm(p_u)


def test_fluxes_telescope(orc):
    """With no Dirichlet wall the volume integral of L p vanishes: every
    interior face flux enters two cells with opposite signs."""
    nx, ny, nz = 5, 4, 9
    h = thicknesses(nz, 8)
    p = np.random.default_rng(9).uniform(-1, 1, (nz, ny, nx))
    for bcs in [(PER, PER, NEU), (NEU, NEU, NEU), (PER, NEU, NEU)]:
        lp = orc.laplacian(p, 0.3, 0.4, None, NEU, bc_x=bcs[0], bc_y=bcs[1], dz_cells=h)
        s = (h[:, None, None] * lp).sum()
        assert abs(s) <= 1e-12 * (h[:, None, None] * np.abs(lp)).sum(), (bcs, s)


@pytest.mark.parametrize("mutation", ["h_face", "h_mean"])
def test_stretched_planted_mistakes_are_caught(orc, mutation):
    nx, ny, nz = 4, 3, 6
    h = thicknesses(nz, 11)
    f = np.random.default_rng(12).uniform(-1, 1, (nz, ny, nx))
    bcs = (PER, NEU, NEU)
    ref, _ = dense_solve(f, 0.2, 0.3, h, bcs)
    p = orc.solve(f, 0.2, 0.3, None, NEU, bc_x=bcs[0], bc_y=bcs[1], dz_cells=h,
                  mutation=mutation)
    assert np.linalg.norm(p - ref) / np.linalg.norm(ref) > 1e-6
