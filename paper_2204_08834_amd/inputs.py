"""Seeded synthetic right-hand sides for the pressure Poisson solve.

Shared by the tests, the benchmark and the smoke check; it holds none of the
solver's arithmetic (no transforms of the solve, no eigenvalues, no
tridiagonal work) and imports neither the oracle nor the GPU binding.

The right-hand side of the Poisson equation of the projection step
(FluTAS, Section 3.3, eqn:poisson) is the discrete divergence of a provisional
face-centred velocity on the marker-and-cell grid of Section 3; the scale
rho_0/dt is taken as 1.  Conventions:

* arrays are float64, shape (nz, ny, nx), x fastest;
* u[k,j,i] sits on the east face x=(i+1)dx, v[k,j,i] on y=(j+1)dy and
  w[k,j,i] on z=(k+1)dz;
* x and y are periodic; with walls in z, w on the top wall (k = nz-1) is set
  to zero and the bottom wall flux is zero;
* D u = (u_i - u_{i-1})/dx + (v_j - v_{j-1})/dy + (w_k - w_{k-1})/dz at the
  cell centres; the result is made zero-mean in FP64.

The workloads stand in for the paper's runs by shape class (the paper's own
flow fields are not available): a triply periodic (2 pi)^3 box as in the
emulsion-in-HIT case, and a 2:2:1 box with walls in z as in the two-layer
Rayleigh-Benard case.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC = 0
NEUMANN = 1


@dataclass
class Problem:
    """One Poisson problem: grid, spacings, z boundary and its right-hand side."""
    name: str
    nx: int
    ny: int
    nz: int
    Lx: float
    Ly: float
    Lz: float
    bc_z: int
    seed: int
    recipe: str
    f: np.ndarray | None = field(default=None, repr=False)

    @property
    def dx(self):
        return self.Lx / self.nx

    @property
    def dy(self):
        return self.Ly / self.ny

    @property
    def dz(self):
        return self.Lz / self.nz

    @property
    def npoints(self):
        return self.nx * self.ny * self.nz

    def spacings(self):
        return self.dx, self.dy, self.dz


# ----------------------------------------------------------------------------
# discrete divergence on the MAC grid (problem definition, not the solver)
# ----------------------------------------------------------------------------
def divergence(u, v, w, dx, dy, dz, bc_z):
    """Cell-centred divergence of face velocities (see module docstring)."""
    d = (u - np.roll(u, 1, axis=2)) / dx
    d += (v - np.roll(v, 1, axis=1)) / dy
    if bc_z == PERIODIC:
        d += (w - np.roll(w, 1, axis=0)) / dz
    else:
        wm = np.empty_like(w)
        wm[0] = 0.0            # bottom wall: no flux
        wm[1:] = w[:-1]
        d += (w - wm) / dz
    return d


def _zero_mean(f):
    return f - f.mean(dtype=np.float64)


def uniform_velocity(nx, ny, nz, bc_z, seed):
    """Face velocities u, v, w ~ U(-1,1) drawn in that order; w on the top
    wall set to 0 for walls."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    u = rng.uniform(-1.0, 1.0, shape)
    v = rng.uniform(-1.0, 1.0, shape)
    w = rng.uniform(-1.0, 1.0, shape)
    if bc_z == NEUMANN:
        w[nz - 1] = 0.0
    return u, v, w


def uniform_velocity_rhs(nx, ny, nz, Lx, Ly, Lz, bc_z, seed):
    """Divergence of uniform_velocity (made zero-mean)."""
    u, v, w = uniform_velocity(nx, ny, nz, bc_z, seed)
    f = divergence(u, v, w, Lx / nx, Ly / ny, Lz / nz, bc_z)
    return _zero_mean(f)


def two_layer_rhs(nx, ny, nz, Lx, Ly, Lz, seed, delta=0.01, contrast=3.0, noise=0.05):
    """Divergence of u/rho_face with a two-layer density (walls in z).

    rho(z) = 1 + contrast*(1 + tanh((z - Lz/2)/delta))/2 at the cell centres
    plus per-cell U(-noise, noise); the face density is the mean of the two
    adjacent cells.  Draw order: u, v, w, then the density noise.
    """
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    u = rng.uniform(-1.0, 1.0, shape)
    v = rng.uniform(-1.0, 1.0, shape)
    w = rng.uniform(-1.0, 1.0, shape)
    w[nz - 1] = 0.0
    dz = Lz / nz
    zc = (np.arange(nz) + 0.5) * dz
    rho_z = 1.0 + contrast * (1.0 + np.tanh((zc - 0.5 * Lz) / delta)) / 2.0
    rho = rho_z[:, None, None] + rng.uniform(-noise, noise, shape)
    rho_u = 0.5 * (rho + np.roll(rho, -1, axis=2))   # face between i and i+1
    rho_v = 0.5 * (rho + np.roll(rho, -1, axis=1))
    rho_w = np.empty_like(rho)
    rho_w[:-1] = 0.5 * (rho[:-1] + rho[1:])
    rho_w[-1] = rho[-1]                               # top wall, w = 0 there
    f = divergence(u / rho_u, v / rho_v, w / rho_w, Lx / nx, Ly / ny, dz, NEUMANN)
    return _zero_mean(f)


def spectral_velocity_rhs(nx, ny, nz, Lx, Ly, Lz, bc_z, seed, smax, slope=-5.0 / 3.0):
    """Divergence of a random-phase velocity with an s^slope shell spectrum.

    Wavevectors k = 2 pi (a/Lx, b/Ly, c/Lz) with integer a, b, c (the field is
    periodic in z with period Lz for the synthesis); shell s = round(|k|/k0),
    k0 = 2 pi / Lx, for s = 1..smax.  Shell energy is proportional to s^slope,
    spread evenly over the shell's modes; each mode's energy is split 50/50
    between a solenoidal part (orthogonal to k) and a potential part (along k),
    both with random phases.  Each velocity component is sampled on its own
    face position.  Random numbers come from one generator per kz plane,
    seeded (seed, plane).  With walls, w on the top wall is set to zero.
    """
    import scipy.fft as sfft
    import sys

    # large grids take minutes: report progress on stderr as the synthesis goes
    verbose = nx * ny * nz >= (1 << 28)

    def note(msg):
        if verbose:
            print(f"[inputs] spectral synthesis {nx}x{ny}x{nz}: {msg}", file=sys.stderr,
                  flush=True)

    nxh = nx // 2 + 1
    k0 = 2.0 * math.pi / Lx
    ax = np.fft.rfftfreq(nx, d=1.0 / nx)            # integer frequencies
    ay = np.fft.fftfreq(ny, d=1.0 / ny)
    az = np.fft.fftfreq(nz, d=1.0 / nz)
    kx = 2.0 * math.pi * ax / Lx
    ky = 2.0 * math.pi * ay / Ly
    kz = 2.0 * math.pi * az / Lz

    # modes per shell over the full (two-sided) spectrum
    counts = np.zeros(smax + 1, dtype=np.float64)
    kxfull = 2.0 * math.pi * np.fft.fftfreq(nx, d=1.0 / nx) / Lx
    kxy2 = kxfull[None, :] ** 2 + ky[:, None] ** 2
    for c in range(nz):
        s = np.rint(np.sqrt(kxy2 + kz[c] ** 2) / k0).astype(np.int64)
        s = s[(s >= 1) & (s <= smax)]
        counts += np.bincount(s, minlength=smax + 1)[: smax + 1]
    shells = np.arange(smax + 1, dtype=np.float64)
    e_mode = np.zeros(smax + 1)
    valid = counts > 0
    e_mode[valid] = shells[valid] ** slope / counts[valid]
    e_mode[0] = 0.0

    dx, dy, dz = Lx / nx, Ly / ny, Lz / nz
    # face offsets relative to the grid index position (i*dx, j*dy, k*dz)
    shifts = ((dx, 0.5 * dy, 0.5 * dz), (0.5 * dx, dy, 0.5 * dz), (0.5 * dx, 0.5 * dy, dz))
    spec = [np.zeros((nz, ny, nxh), dtype=np.complex128) for _ in range(3)]
    kxy_x = np.broadcast_to(kx[None, :], (ny, nxh))
    kxy_y = np.broadcast_to(ky[:, None], (ny, nxh))
    for c in range(nz):
        rng = np.random.default_rng([seed, c])
        kk = np.stack([kxy_x, kxy_y, np.full((ny, nxh), kz[c])])
        kmag = np.sqrt((kk ** 2).sum(axis=0))
        s = np.rint(kmag / k0).astype(np.int64)
        amp = np.where((s >= 1) & (s <= smax), np.sqrt(e_mode[np.clip(s, 0, smax)]), 0.0)
        khat = kk / np.where(kmag > 0, kmag, 1.0)
        a = rng.standard_normal((3, ny, nxh)) + 1j * rng.standard_normal((3, ny, nxh))
        a -= (a * khat).sum(axis=0) * khat                 # solenoidal: orthogonal to k
        an = np.sqrt((np.abs(a) ** 2).sum(axis=0))
        a *= np.where(an > 0, 1.0 / np.where(an > 0, an, 1.0), 0.0)
        theta = rng.uniform(0.0, 2.0 * math.pi, (ny, nxh))
        pot = np.exp(1j * theta) * khat                    # potential: along k
        vec = (a + pot) * (amp * math.sqrt(0.5))
        for comp in range(3):
            sx, sy, sz = shifts[comp]
            phase = np.exp(1j * (kk[0] * sx + kk[1] * sy + kk[2] * sz))
            spec[comp][c] = vec[comp] * phase
        if (c + 1) % 64 == 0:
            note(f"modes of {c + 1}/{nz} kz planes")

    norm = nx * ny * nz
    vel = []
    for comp in range(3):
        field_c = sfft.irfftn(spec[comp], s=(nz, ny, nx), axes=(0, 1, 2), workers=-1) * norm
        spec[comp] = None
        vel.append(field_c)
        note(f"velocity component {comp + 1}/3 transformed")
    u, v, w = vel
    rms = math.sqrt(float((u * u).mean() + (v * v).mean() + (w * w).mean()) / 3.0)
    if rms > 0:
        u /= rms
        v /= rms
        w /= rms
    if bc_z == NEUMANN:
        w[nz - 1] = 0.0
    f = divergence(u, v, w, dx, dy, dz, bc_z)
    return _zero_mean(f)


def spectral_velocity_rhs_torch(nx, ny, nz, Lx, Ly, Lz, bc_z, seed, smax, slope=-5.0 / 3.0,
                                device="cuda", chunk=32):
    """The recipe of spectral_velocity_rhs synthesised on a GPU with torch
    (for grids whose synthesis on the host takes minutes): the same shells,
    shell energies, solenoidal / potential split, face sampling, rms
    normalisation, top-wall w = 0 and zero-mean divergence; random numbers
    from one torch generator seeded with `seed`, drawn plane chunk by plane
    chunk (a different realisation of the recipe than the host version's).
    Returns the right-hand side as a float64 tensor on `device`."""
    import torch

    f64, c128 = torch.float64, torch.complex128
    dev = torch.device(device)
    nxh = nx // 2 + 1
    k0 = 2.0 * math.pi / Lx
    kx = 2.0 * math.pi * torch.fft.rfftfreq(nx, d=1.0 / nx, dtype=f64, device=dev) / Lx
    kxf = 2.0 * math.pi * torch.fft.fftfreq(nx, d=1.0 / nx, dtype=f64, device=dev) / Lx
    ky = 2.0 * math.pi * torch.fft.fftfreq(ny, d=1.0 / ny, dtype=f64, device=dev) / Ly
    kz = 2.0 * math.pi * torch.fft.fftfreq(nz, d=1.0 / nz, dtype=f64, device=dev) / Lz
    # modes per shell over the full two-sided spectrum
    counts = torch.zeros(smax + 1, dtype=f64, device=dev)
    kxy2 = kxf[None, :] ** 2 + ky[:, None] ** 2
    for c in range(nz):
        sh = torch.round(torch.sqrt(kxy2 + kz[c] ** 2) / k0).to(torch.int64)
        sh = sh[(sh >= 1) & (sh <= smax)]
        counts += torch.bincount(sh, minlength=smax + 1)[: smax + 1].to(f64)
    shells = torch.arange(smax + 1, dtype=f64, device=dev)
    e_mode = torch.where(counts > 0, shells.clamp(min=1.0) ** slope / counts.clamp(min=1.0),
                         torch.zeros_like(counts))
    e_mode[0] = 0.0
    dx, dy, dz = Lx / nx, Ly / ny, Lz / nz
    shifts = ((dx, 0.5 * dy, 0.5 * dz), (0.5 * dx, dy, 0.5 * dz), (0.5 * dx, 0.5 * dy, dz))
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    spec = [torch.zeros((nz, ny, nxh), dtype=c128, device=dev) for _ in range(3)]
    KX = kx[None, None, :].expand(1, ny, nxh)
    KY = ky[None, :, None].expand(1, ny, nxh)
    for c0 in range(0, nz, chunk):
        c1 = min(nz, c0 + chunk)
        m = c1 - c0
        KZ = kz[c0:c1, None, None].expand(m, ny, nxh)
        kk = torch.stack([KX.expand(m, ny, nxh), KY.expand(m, ny, nxh), KZ])
        kmag = torch.sqrt((kk ** 2).sum(0))
        sh = torch.round(kmag / k0).to(torch.int64)
        ok = (sh >= 1) & (sh <= smax)
        amp = torch.where(ok, torch.sqrt(e_mode[sh.clamp(0, smax)]), torch.zeros_like(kmag))
        khat = kk / torch.where(kmag > 0, kmag, torch.ones_like(kmag))
        a = torch.complex(torch.randn((3, m, ny, nxh), generator=gen, dtype=f64, device=dev),
                          torch.randn((3, m, ny, nxh), generator=gen, dtype=f64, device=dev))
        a = a - (a * khat).sum(0) * khat
        an = torch.sqrt((a.abs() ** 2).sum(0))
        a = a * torch.where(an > 0, 1.0 / torch.where(an > 0, an, torch.ones_like(an)),
                            torch.zeros_like(an))
        theta = torch.rand((m, ny, nxh), generator=gen, dtype=f64, device=dev) * (2.0 * math.pi)
        pot = torch.exp(1j * theta) * khat
        vec = (a + pot) * (amp * math.sqrt(0.5))
        for comp in range(3):
            sx, sy, sz = shifts[comp]
            phase = torch.exp(1j * (kk[0] * sx + kk[1] * sy + kk[2] * sz))
            spec[comp][c0:c1] = vec[comp] * phase
        del kk, kmag, sh, ok, amp, khat, a, an, theta, pot, vec
    norm = nx * ny * nz
    vel = []
    for comp in range(3):
        vel.append(torch.fft.irfftn(spec[comp], s=(nz, ny, nx), dim=(0, 1, 2)) * norm)
        spec[comp] = None
    u, v, w = vel
    rms = math.sqrt(float((u * u).mean() + (v * v).mean() + (w * w).mean()) / 3.0)
    if rms > 0:
        u /= rms
        v /= rms
        w /= rms
    if bc_z == NEUMANN:
        w[nz - 1] = 0.0
    f = (u - torch.roll(u, 1, dims=2)) / dx
    del u
    f += (v - torch.roll(v, 1, dims=1)) / dy
    del v
    if bc_z == PERIODIC:
        f += (w - torch.roll(w, 1, dims=0)) / dz
    else:
        wm = torch.empty_like(w)
        wm[0] = 0.0
        wm[1:] = w[:-1]
        f += (w - wm) / dz
    return f - f.mean(dtype=f64)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def _mk(name, nx, ny, nz, Lx, Ly, Lz, bc_z, seed, recipe):
    return Problem(name, nx, ny, nz, Lx, Ly, Lz, bc_z, seed, recipe)


TWO_PI = 2.0 * math.pi

WORKLOADS = {
    # 32^3 unit box, walls in z, U(-1,1) velocities, seed 42
    "walls32": lambda: _mk("walls32", 32, 32, 32, 1.0, 1.0, 1.0, NEUMANN, 42, "uniform"),
    # 256^3 (2 pi)^3 triply periodic, k^-5/3 spectral velocity, shells 1..85
    "hit256": lambda: _mk("hit256", 256, 256, 256, TWO_PI, TWO_PI, TWO_PI, PERIODIC, 2,
                          "spectral:85"),
    # 512x512x256, 2:2:1, walls in z, two-layer density
    "rb512": lambda: _mk("rb512", 512, 512, 256, 2.0, 2.0, 1.0, NEUMANN, 3, "two_layer"),
    # 1024x1024x512, 2:2:1, walls in z, k^-5/3 spectral velocity, shells 1..341
    "rb1024": lambda: _mk("rb1024", 1024, 1024, 512, 2.0, 2.0, 1.0, NEUMANN, 5,
                          "spectral:341"),
}


def batch_mixed64():
    """64 problems: 24 x 64^3 periodic (2 pi)^3, 24 x 96x96x48 walls (2:2:1),
    16 x 128x128x64 walls (2:2:1); seeds 1000+b, U(-1,1) face velocities."""
    probs = []
    b = 0
    for _ in range(24):
        probs.append(_mk(f"b{b}_p64", 64, 64, 64, TWO_PI, TWO_PI, TWO_PI, PERIODIC, 1000 + b,
                         "uniform"))
        b += 1
    for _ in range(24):
        probs.append(_mk(f"b{b}_w96", 96, 96, 48, 2.0, 2.0, 1.0, NEUMANN, 1000 + b, "uniform"))
        b += 1
    for _ in range(16):
        probs.append(_mk(f"b{b}_w128", 128, 128, 64, 2.0, 2.0, 1.0, NEUMANN, 1000 + b,
                         "uniform"))
        b += 1
    return probs


def make_rhs(prob: Problem) -> np.ndarray:
    """Generate (and cache on the Problem) the right-hand side."""
    if prob.f is not None:
        return prob.f
    r = prob.recipe
    if r == "uniform":
        f = uniform_velocity_rhs(prob.nx, prob.ny, prob.nz, prob.Lx, prob.Ly, prob.Lz,
                                 prob.bc_z, prob.seed)
    elif r == "two_layer":
        f = two_layer_rhs(prob.nx, prob.ny, prob.nz, prob.Lx, prob.Ly, prob.Lz, prob.seed)
    elif r.startswith("spectral:"):
        smax = int(r.split(":")[1])
        f = spectral_velocity_rhs(prob.nx, prob.ny, prob.nz, prob.Lx, prob.Ly, prob.Lz,
                                  prob.bc_z, prob.seed, smax)
    else:
        raise ValueError(f"unknown recipe {r}")
    prob.f = f
    return f


def workload(name: str, with_rhs: bool = True) -> Problem:
    p = WORKLOADS[name]()
    if with_rhs:
        make_rhs(p)
    return p


def scaled(name: str, nx: int, ny: int, nz: int, seed: int | None = None) -> Problem:
    """Same shape class (box, boundary, recipe) as a named workload, other sizes."""
    base = WORKLOADS[name]()
    recipe = base.recipe
    if recipe.startswith("spectral:"):
        recipe = f"spectral:{max(1, min(nx, ny, nz) // 3)}"
    p = Problem(f"{name}@{nx}x{ny}x{nz}", nx, ny, nz, base.Lx, base.Ly, base.Lz, base.bc_z,
                base.seed if seed is None else seed, recipe)
    make_rhs(p)
    return p


def tanh_cells(nz, Lz=1.0, beta=2.0):
    """Cell thicknesses of a wall-bounded axis clustered at both walls: the
    faces sit at z_f(t) = Lz (1 + tanh(beta (2t - 1)) / tanh(beta)) / 2,
    t = k / nz (the usual tanh stretching of channel and convection grids;
    beta = 0 is the uniform grid)."""
    t = np.arange(nz + 1) / nz
    if beta == 0:
        zf = Lz * t
    else:
        zf = Lz * (1.0 + np.tanh(beta * (2.0 * t - 1.0)) / math.tanh(beta)) / 2.0
    return np.diff(zf)


def random_rhs(nx, ny, nz, seed, zero_mean=True):
    """Plain U(-1,1) cell data (not a divergence), for tests of linear algebra."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, (nz, ny, nx))
    return _zero_mean(f) if zero_mean else f
