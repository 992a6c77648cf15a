/*
 * poisson_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for the pressure Poisson solve of the
 * two-fluid projection method (FluTAS, arXiv 2204.08834).  It exists to check
 * the GPU path; nothing in the product library links, calls or includes it.
 * Only the tests, the package's smoke check and the CPU-baseline leg of the
 * benchmark may load it.
 *
 * What it computes (Section 3.3 "Pressure correction algorithm", equation
 * eqn:poisson, and Section 3.3.1 "Poisson solver"):
 *
 *   the unique zero-mean p with  L p = f - mean(f),
 *
 * where L is the second-order finite-difference Laplacian on the uniform
 * marker-and-cell grid of Section 3 (pressure at cell centres; seven
 * non-zero diagonals, Section 3.3.1).  Each axis is periodic or bounded by
 * walls on the end faces of the cells with a homogeneous condition: zero
 * normal gradient (the wall condition stated after eqn:corr; the ghost value
 * mirrors the wall cell) or zero value (the ghost value is the negated wall
 * cell) -- the homogeneous pressure conditions the solver of Section 3.3.1
 * covers with its Fourier-based expansions.  With a zero-value wall anywhere
 * the system is regular: nothing is removed and p is not shifted.
 *
 * How (the eigen-expansion of Section 3.3.1, taken in its steps):
 *   1. remove the mean of f (when the constant is in the null space);
 *   2. forward expansion along x, then along y: a discrete Fourier transform
 *      for a periodic axis, the cosine or sine basis of the wall condition
 *      otherwise (textbook O(n^2) sums, no symmetry shortcuts);
 *   3. per mode pair (mx,my): walls in z -> tridiagonal system along z solved
 *      by Gauss elimination without pivoting (Thomas); periodic -> DFT along
 *      z and division by the eigenvalue of the 3-D operator;
 *   4. inverse expansions along y then x, keep the real part;
 *   5. remove the mean of p (the gauge; the paper leaves it open).
 *
 * Eigenvalues of the periodic 3-point operator (not printed in the paper;
 * they follow from applying the stencil to exp(2 pi i m n / N)):
 *   lambda(m) = -(4/h^2) sin^2(pi m / N).
 *
 * Parity pins: see the tests (closed-form discrete eigenmodes, dense LU on
 * small grids, zero mean, residual at machine precision, projection
 * invariant, symmetries, 1-D reductions to DCT-II).
 *
 * Also the projection around the solve (oracle_divergence, oracle_correct):
 * the right-hand side alpha D u of the face velocities and the velocity
 * update u -= beta G psi.
 *
 * A "mutation" argument plants one known mistake at a time so the tests can
 * show that the pins catch it.  mutation = 0 is the oracle.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PERIODIC 0
#define ORC_NEUMANN 1
#define ORC_DIRICHLET 2

/* mutations (test-only planted mistakes) */
#define MUT_NONE 0
#define MUT_FWD_SIGN_X 1      /* forward x DFT uses exp(+i..), inverse unchanged */
#define MUT_WALL_ROW 2        /* wall rows use the interior diagonal */
#define MUT_HALF_ANGLE 3      /* eigenvalue with sin^2(pi m/(2N)) */
#define MUT_SWAP_DXDY 4       /* dx and dy exchanged in the eigenvalues */
#define MUT_NO_NORM_Y 5       /* inverse y DFT without 1/ny */
#define MUT_NO_GAUGE 6        /* final mean removal skipped, zero mode pinned at k=nz-1 */
#define MUT_DROP_Z 7          /* the z part of the operator dropped (walls) */
#define MUT_OFFDIAG 8         /* off-diagonal of the z system uses 1/dx^2 */
#define MUT_IDX_Y 9           /* y DFT exponent uses (m*j+1) */
#define MUT_DIR_ROW 10        /* Dirichlet wall rows use the Neumann diagonal */
#define MUT_COS_SHIFT 11      /* cosine basis without the half-cell shift */
#define MUT_SIN_INDEX 12      /* sine basis index k instead of k+1 */
/* planted mistakes of the operator and residual evaluation */
#define MUT_RES_NO_SQRT 13    /* relative L2 residual reported without the square root */
#define MUT_LAP_DIR_X 14      /* Dirichlet x wall takes the mirrored (Neumann) ghost in L */
#define MUT_LAP_DIR_Y 15      /* Dirichlet y wall takes the mirrored (Neumann) ghost in L */
#define MUT_RES_NO_MEAN 16    /* residual keeps the mean of f on a singular problem */
#define MUT_RES_MEAN_DIR 17   /* residual removes the mean of f despite a Dirichlet wall */
/* planted mistakes of the stretched-z solve */
#define MUT_H_FACE 18         /* distance between cell centres k, k+1 taken as h[k] */
#define MUT_H_MEAN 19         /* plain (unweighted) mean of f removed and of p as the gauge */

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* lambda(m) = -(4/h^2) sin^2(pi m/N): eigenvalue of the periodic
 * three-point second difference on N points of spacing h. */
static double eig_periodic(int m, int n, double h, int mutation)
{
    double ang = (mutation == MUT_HALF_ANGLE) ? ORC_PI * m / (2.0 * n) : ORC_PI * m / n;
    double s = sin(ang);
    return -4.0 / (h * h) * s * s;
}

/* pairwise (cascade) sum for the mean */
static double pairwise_sum(const double *v, long n)
{
    if (n <= 32) {
        double s = 0.0;
        for (long i = 0; i < n; ++i) s += v[i];
        return s;
    }
    long h = n / 2;
    return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

/* w[t] = exp(sign * 2 pi i t / n), t = 0..n-1 */
static void twiddles(int n, int sign, double complex *w)
{
    for (int t = 0; t < n; ++t) {
        double a = sign * 2.0 * ORC_PI * (double)t / (double)n;
        w[t] = cos(a) + I * sin(a);
    }
}

/* Textbook DFT of one strided line: out[m] = sum_i in[i] * w[(m*i) mod n]. */
static void dft_line(int n, const double complex *w, const double complex *in,
                     long stride, double complex *out, int idx_mut)
{
    for (int m = 0; m < n; ++m) {
        double complex acc = 0.0;
        for (int i = 0; i < n; ++i) {
            long t = ((long)m * i + (idx_mut ? 1 : 0)) % n;
            acc += in[(long)i * stride] * w[t];
        }
        out[m] = acc;
    }
}

/* Apply a DFT (sign -1 forward, +1 inverse, scale applied to the output)
 * along axis 0 (x), 1 (y) or 2 (z) of a complex (nz,ny,nx) array. */
static void dft_axis(double complex *a, int nx, int ny, int nz, int axis, int sign,
                     double scale, int mutation)
{
    int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    long stride = axis == 0 ? 1 : (axis == 1 ? nx : (long)nx * ny);
    long nlines = (long)nx * ny * nz / n;
    int sgn = sign;
    if (axis == 0 && sign < 0 && mutation == MUT_FWD_SIGN_X) sgn = +1;
    int idx_mut = (axis == 1 && sign < 0 && mutation == MUT_IDX_Y);
    double complex *w = malloc(sizeof(double complex) * n);
    twiddles(n, sgn, w);
#pragma omp parallel
    {
        double complex *in = malloc(sizeof(double complex) * n);
        double complex *out = malloc(sizeof(double complex) * n);
#pragma omp for schedule(static)
        for (long l = 0; l < nlines; ++l) {
            long base;
            if (axis == 0) {
                base = l * nx;
            } else if (axis == 1) {
                long k = l / nx, i = l % nx;
                base = k * (long)nx * ny + i;
            } else {
                base = l; /* l = j*nx + i */
            }
            for (int t = 0; t < n; ++t) in[t] = a[base + (long)t * stride];
            dft_line(n, w, in, 1, out, idx_mut);
            for (int t = 0; t < n; ++t) a[base + (long)t * stride] = out[t] * scale;
        }
        free(in);
        free(out);
    }
    free(w);
}

/* Basis functions of the cell-centred three-point operator with a wall on
 * each end face (Section 3: pressure at cell centres; the walls sit on the
 * faces i = -1/2 and i = n - 1/2):
 *   Neumann (mirrored ghost):  phi_k(i) = cos(pi k (i + 1/2) / n),
 *                              lambda_k = -(4/h^2) sin^2(pi k / (2n));
 *   Dirichlet (negated ghost): phi_k(i) = sin(pi (k+1) (i + 1/2) / n),
 *                              lambda_k = -(4/h^2) sin^2(pi (k+1) / (2n)),
 * k = 0..n-1.  Both follow from applying the stencil to phi_k: the ghost
 * value at a wall is phi_k(-1) = phi_k(0) (cosines) or -phi_k(0) (sines).
 * The bases are orthogonal with sum_i phi_k(i)^2 = n/2, except n for k = 0
 * (cosines) and for k = n-1 (sines). */
static double basis(int type, int k, int i, int n, int mutation)
{
    if (type == ORC_NEUMANN) {
        double x = (mutation == MUT_COS_SHIFT) ? (double)i : i + 0.5;
        return cos(ORC_PI * k * x / n);
    }
    int kk = (mutation == MUT_SIN_INDEX) ? k : k + 1;
    return sin(ORC_PI * kk * (i + 0.5) / n);
}

static double basis_norm2(int type, int k, int n)
{
    if (type == ORC_NEUMANN) return k == 0 ? (double)n : 0.5 * n;
    return k == n - 1 ? (double)n : 0.5 * n;
}

static double eig_wall(int type, int k, int n, double h)
{
    double ang = (type == ORC_NEUMANN) ? ORC_PI * k / (2.0 * n) : ORC_PI * (k + 1) / (2.0 * n);
    double s = sin(ang);
    return -4.0 / (h * h) * s * s;
}

/* Expansion in one of the wall bases along axis 0 (x) or 1 (y) of a complex
 * (nz,ny,nx) array, applied to real and imaginary parts alike (the bases are
 * real): forward c_k = sum_i a_i phi_k(i); inverse a_i = sum_k c_k phi_k(i) /
 * ||phi_k||^2.  Textbook O(n^2) sums. */
static void wall_axis(double complex *a, int nx, int ny, int nz, int axis, int type,
                      int inverse, int mutation)
{
    int n = axis == 0 ? nx : ny;
    long stride = axis == 0 ? 1 : nx;
    long nlines = (long)nx * ny * nz / n;
    double *tab = malloc(sizeof(double) * (size_t)n * n); /* tab[k*n + i] = phi_k(i) */
    for (int k = 0; k < n; ++k)
        for (int i = 0; i < n; ++i) tab[(long)k * n + i] = basis(type, k, i, n, mutation);
#pragma omp parallel
    {
        double complex *in = malloc(sizeof(double complex) * n);
#pragma omp for schedule(static)
        for (long l = 0; l < nlines; ++l) {
            long base;
            if (axis == 0) {
                base = l * nx;
            } else {
                long k = l / nx, i = l % nx;
                base = k * (long)nx * ny + i;
            }
            for (int t = 0; t < n; ++t) in[t] = a[base + (long)t * stride];
            for (int o = 0; o < n; ++o) {
                double complex acc = 0.0;
                if (!inverse) {
                    for (int i = 0; i < n; ++i) acc += in[i] * tab[(long)o * n + i];
                } else {
                    for (int k = 0; k < n; ++k)
                        acc += in[k] * tab[(long)k * n + o] / basis_norm2(type, k, n);
                }
                a[base + (long)o * stride] = acc;
            }
        }
        free(in);
    }
    free(tab);
}

/* eigenvalue of mode m of the three-point operator along one axis */
static double eig_axis(int bc, int m, int n, double h, int mutation)
{
    return bc == ORC_PERIODIC ? eig_periodic(m, n, h, mutation) : eig_wall(bc, m, n, h);
}

/* Thomas algorithm (Gauss elimination without pivoting) for
 *   lo[k] x[k-1] + di[k] x[k] + up[k] x[k+1] = d[k],  k = 0..n-1,
 * real coefficients, complex right-hand side, solved in place. */
static void thomas(int n, const double *lo, const double *di, const double *up,
                   double complex *d, double *cp)
{
    if (n <= 0) return;
    cp[0] = up[0] / di[0];
    d[0] = d[0] / di[0];
    for (int k = 1; k < n; ++k) {
        double piv = di[k] - lo[k] * cp[k - 1];
        cp[k] = up[k] / piv;
        d[k] = (d[k] - lo[k] * d[k - 1]) / piv;
    }
    for (int k = n - 2; k >= 0; --k) d[k] -= cp[k] * d[k + 1];
}

/* z solve for wall-bounded boxes, one (mx,my) column of the x-y spectrum.
 * Rows (units 1/dz^2): a p[k-1] + (lam - 2a) p[k] + a p[k+1] = g[k]; at a
 * wall the ghost value is p[0] (Neumann, mirrored) or -p[0] (Dirichlet,
 * negated), which turns the wall rows into (lam - a) p[0] + a p[1] or
 * (lam - 3a) p[0] + a p[1] (likewise at the top).
 * For the singular column (Neumann, zero wavenumber) the value at k=0 is
 * pinned to zero, the redundant first row is dropped, and the column mean is
 * removed afterwards. */
static void zsolve_walls(int nz, double dz, double lam, int singular, double complex *g,
                         double *lo, double *di, double *up, double *cp, int mutation,
                         double dx, int bc_z)
{
    double a = 1.0 / (dz * dz);
    if (mutation == MUT_OFFDIAG) a = 1.0 / (dx * dx);
    double two_a = 2.0 / (dz * dz);
    if (mutation == MUT_DROP_Z) { a = 0.0; two_a = 0.0; }
    for (int k = 0; k < nz; ++k) {
        lo[k] = (k > 0) ? a : 0.0;
        up[k] = (k < nz - 1) ? a : 0.0;
        double nb = 0.0; /* number of real (non-ghost) neighbours times a */
        if (k > 0) nb += a;
        if (k < nz - 1) nb += a;
        di[k] = lam - nb;
        if (bc_z == ORC_DIRICHLET && mutation != MUT_DIR_ROW) {
            if (k == 0) di[k] -= 2.0 * a;       /* ghost -p[0]: -2a - a */
            if (k == nz - 1) di[k] -= 2.0 * a;  /* ghost -p[nz-1] */
        }
        if (mutation == MUT_WALL_ROW) di[k] = lam - two_a;
        if (mutation == MUT_DROP_Z) di[k] = lam;
    }
    if (!singular) {
        thomas(nz, lo, di, up, g, cp);
        return;
    }
    int pin = (mutation == MUT_NO_GAUGE) ? nz - 1 : 0;
    if (nz == 1) { g[0] = 0.0; return; }
    if (pin == 0) {
        /* unknowns p[1..nz-1], p[0] = 0 */
        thomas(nz - 1, lo + 1, di + 1, up + 1, g + 1, cp);
        g[0] = 0.0;
    } else {
        /* unknowns p[0..nz-2], p[nz-1] = 0 */
        thomas(nz - 1, lo, di, up, g, cp);
        g[nz - 1] = 0.0;
    }
    if (mutation != MUT_NO_GAUGE) {
        double complex s = 0.0;
        for (int k = 0; k < nz; ++k) s += g[k];
        s /= nz;
        for (int k = 0; k < nz; ++k) g[k] -= s;
    }
}

/*
 * oracle_solve_bc: the full solve with a boundary condition per axis and an
 * optional planted mistake.
 *   f, p: (nz,ny,nx) C-order (x fastest) double arrays, p written.
 *   bc_x, bc_y, bc_z: 0 periodic, 1 walls with homogeneous Neumann (zero
 *   normal gradient), 2 walls with homogeneous Dirichlet (zero value on the
 *   wall face); walls sit on the end faces of the cells.
 *   When no axis is Dirichlet the operator has the constant null vector: the
 *   mean of f is removed (and reported) and p is made zero-mean.  Otherwise
 *   the system is regular, nothing is removed and rhs_mean receives 0.
 *   rhs_mean (nullable), max_imag (nullable): max|Im| / max|Re| before the
 *   real part is taken.
 * Returns 0 on success, -1 on bad arguments or allocation failure.
 */
int oracle_solve_bc(int nx, int ny, int nz, double dx, double dy, double dz, int bc_x,
                    int bc_y, int bc_z, const double *f, double *p, double *rhs_mean,
                    double *max_imag, int mutation)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0) || !(dy > 0) || !(dz > 0) || !f || !p)
        return -1;
    if (bc_x < 0 || bc_x > 2 || bc_y < 0 || bc_y > 2 || bc_z < 0 || bc_z > 2) return -1;
    const int singular_problem =
        bc_x != ORC_DIRICHLET && bc_y != ORC_DIRICHLET && bc_z != ORC_DIRICHLET;
    long n = (long)nx * ny * nz;
    double complex *a = malloc(sizeof(double complex) * n);
    if (!a) return -1;

    /* 1. remove the mean (only where the constant is in the null space) */
    double mean = singular_problem ? pairwise_sum(f, n) / (double)n : 0.0;
    if (rhs_mean) *rhs_mean = mean;
    for (long t = 0; t < n; ++t) a[t] = f[t] - mean;

    /* 2. forward expansions along x and y */
    if (bc_x == ORC_PERIODIC)
        dft_axis(a, nx, ny, nz, 0, -1, 1.0, mutation);
    else
        wall_axis(a, nx, ny, nz, 0, bc_x, 0, mutation);
    if (bc_y == ORC_PERIODIC)
        dft_axis(a, nx, ny, nz, 1, -1, 1.0, mutation);
    else
        wall_axis(a, nx, ny, nz, 1, bc_y, 0, mutation);

    double hx = dx, hy = dy;
    if (mutation == MUT_SWAP_DXDY) { hx = dy; hy = dx; }

    /* 3. z-solve per (mx,my) */
    if (bc_z != ORC_PERIODIC) {
#pragma omp parallel
        {
            double complex *g = malloc(sizeof(double complex) * nz);
            double *lo = malloc(sizeof(double) * nz), *di = malloc(sizeof(double) * nz);
            double *up = malloc(sizeof(double) * nz), *cp = malloc(sizeof(double) * nz);
#pragma omp for schedule(static)
            for (long q = 0; q < (long)nx * ny; ++q) {
                int mx = (int)(q % nx), my = (int)(q / nx);
                double lam = eig_axis(bc_x, mx, nx, hx, mutation) +
                             eig_axis(bc_y, my, ny, hy, mutation);
                int singular = singular_problem && mx == 0 && my == 0;
                for (int k = 0; k < nz; ++k) g[k] = a[(long)k * nx * ny + q];
                zsolve_walls(nz, dz, lam, singular, g, lo, di, up, cp, mutation, dx, bc_z);
                for (int k = 0; k < nz; ++k) a[(long)k * nx * ny + q] = g[k];
            }
            free(g); free(lo); free(di); free(up); free(cp);
        }
    } else {
        dft_axis(a, nx, ny, nz, 2, -1, 1.0, mutation);
#pragma omp parallel for schedule(static)
        for (long t = 0; t < n; ++t) {
            int mx = (int)(t % nx);
            int my = (int)((t / nx) % ny);
            int mz = (int)(t / ((long)nx * ny));
            double lam = eig_axis(bc_x, mx, nx, hx, mutation) +
                         eig_axis(bc_y, my, ny, hy, mutation);
            double lz = eig_periodic(mz, nz, dz, mutation);
            if (mutation == MUT_DROP_Z) lz = 0.0;
            lam += lz;
            if (singular_problem && mx == 0 && my == 0 && mz == 0)
                a[t] = 0.0;
            else if (lam == 0.0)
                a[t] = 0.0; /* only reachable with a planted mistake */
            else
                a[t] /= lam;
        }
        dft_axis(a, nx, ny, nz, 2, +1, 1.0 / nz, mutation);
    }

    /* 4. inverse expansions along y then x */
    if (bc_y == ORC_PERIODIC)
        dft_axis(a, nx, ny, nz, 1, +1, mutation == MUT_NO_NORM_Y ? 1.0 : 1.0 / ny, mutation);
    else
        wall_axis(a, nx, ny, nz, 1, bc_y, 1, mutation);
    if (bc_x == ORC_PERIODIC)
        dft_axis(a, nx, ny, nz, 0, +1, 1.0 / nx, mutation);
    else
        wall_axis(a, nx, ny, nz, 0, bc_x, 1, mutation);

    double mre = 0.0, mim = 0.0;
    for (long t = 0; t < n; ++t) {
        p[t] = creal(a[t]);
        double re = fabs(creal(a[t])), im = fabs(cimag(a[t]));
        if (re > mre) mre = re;
        if (im > mim) mim = im;
    }
    if (max_imag) *max_imag = (mre > 0) ? mim / mre : mim;
    free(a);

    /* 5. gauge: zero mean (singular problems only) */
    if (singular_problem && mutation != MUT_NO_GAUGE) {
        double pm = pairwise_sum(p, n) / (double)n;
        for (long t = 0; t < n; ++t) p[t] -= pm;
    }
    return 0;
}

/* the solve with x and y periodic (the original interface) */
int oracle_solve_ex(int nx, int ny, int nz, double dx, double dy, double dz, int bc_z,
                    const double *f, double *p, double *rhs_mean, double *max_imag,
                    int mutation)
{
    if (bc_z != ORC_PERIODIC && bc_z != ORC_NEUMANN) return -1;
    return oracle_solve_bc(nx, ny, nz, dx, dy, dz, ORC_PERIODIC, ORC_PERIODIC, bc_z, f, p,
                           rhs_mean, max_imag, mutation);
}

int oracle_solve(int nx, int ny, int nz, double dx, double dy, double dz, int bc_z,
                 const double *f, double *p, double *rhs_mean, double *max_imag)
{
    return oracle_solve_ex(nx, ny, nz, dx, dy, dz, bc_z, f, p, rhs_mean, max_imag, MUT_NONE);
}

/* neighbour of index i at offset +1 or -1 along an axis of n cells:
 * returns the index and the factor of the ghost value (1 periodic or
 * mirrored, -1 negated at a Dirichlet wall) */
static int nbr(int i, int d, int n, int bc, double *fac)
{
    int j = i + d;
    *fac = 1.0;
    if (j >= 0 && j < n) return j;
    if (bc == ORC_PERIODIC) return (j + n) % n;
    if (bc == ORC_DIRICHLET) *fac = -1.0;
    return i; /* the ghost mirrors (or negates) the wall cell */
}

/*
 * oracle_laplacian_bc: out = L p, the 7-point operator of Section 3 on the
 * MAC grid with per-axis boundaries (0 periodic, 1 Neumann: ghost = wall
 * cell, 2 Dirichlet: ghost = -wall cell).
 */
int oracle_laplacian_bc_mut(int nx, int ny, int nz, double dx, double dy, double dz, int bc_x,
                            int bc_y, int bc_z, const double *p, double *out, int mutation)
{
    if (nx < 1 || ny < 1 || nz < 1 || !p || !out) return -1;
    if (mutation == MUT_LAP_DIR_X && bc_x == ORC_DIRICHLET) bc_x = ORC_NEUMANN;
    if (mutation == MUT_LAP_DIR_Y && bc_y == ORC_DIRICHLET) bc_y = ORC_NEUMANN;
    double ax = 1.0 / (dx * dx), ay = 1.0 / (dy * dy), az = 1.0 / (dz * dz);
#pragma omp parallel for schedule(static)
    for (long kk = 0; kk < (long)nz * ny; ++kk) {
        int k = (int)(kk / ny), j = (int)(kk % ny);
        double fjm, fjp, fkm, fkp;
        int jm = nbr(j, -1, ny, bc_y, &fjm), jp = nbr(j, +1, ny, bc_y, &fjp);
        int km = nbr(k, -1, nz, bc_z, &fkm), kp = nbr(k, +1, nz, bc_z, &fkp);
        for (int i = 0; i < nx; ++i) {
            double fim, fip;
            int im = nbr(i, -1, nx, bc_x, &fim), ip = nbr(i, +1, nx, bc_x, &fip);
#define P(K, J, I) p[((long)(K) * ny + (J)) * nx + (I)]
            double c = P(k, j, i);
            double v = ax * (fip * P(k, j, ip) - 2.0 * c + fim * P(k, j, im)) +
                       ay * (fjp * P(k, jp, i) - 2.0 * c + fjm * P(k, jm, i)) +
                       az * (fkp * P(kp, j, i) - 2.0 * c + fkm * P(km, j, i));
#undef P
            out[((long)k * ny + j) * nx + i] = v;
        }
    }
    return 0;
}

int oracle_laplacian_bc(int nx, int ny, int nz, double dx, double dy, double dz, int bc_x,
                        int bc_y, int bc_z, const double *p, double *out)
{
    return oracle_laplacian_bc_mut(nx, ny, nz, dx, dy, dz, bc_x, bc_y, bc_z, p, out, MUT_NONE);
}

/* x and y periodic; z periodic or Neumann walls (the original interface) */
int oracle_laplacian(int nx, int ny, int nz, double dx, double dy, double dz, int bc_z,
                     const double *p, double *out)
{
    return oracle_laplacian_bc(nx, ny, nz, dx, dy, dz, ORC_PERIODIC, ORC_PERIODIC, bc_z, p, out);
}

/*
 * oracle_residual_bc: r = (f - mean(f)) - L p (the mean is removed only when
 * no axis is Dirichlet, as in the solve), plus the relative L2 and Linf norms
 * ||r|| / ||f - mean(f)||.  r may be NULL.  (_mut: with a planted mistake.)
 */
int oracle_residual_bc_mut(int nx, int ny, int nz, double dx, double dy, double dz, int bc_x,
                           int bc_y, int bc_z, const double *f, const double *p, double *r,
                           double *rel_l2, double *rel_linf, int mutation)
{
    long n = (long)nx * ny * nz;
    double *lp = malloc(sizeof(double) * n);
    if (!lp) return -1;
    if (oracle_laplacian_bc_mut(nx, ny, nz, dx, dy, dz, bc_x, bc_y, bc_z, p, lp, mutation)) {
        free(lp);
        return -1;
    }
    int singular_problem =
        bc_x != ORC_DIRICHLET && bc_y != ORC_DIRICHLET && bc_z != ORC_DIRICHLET;
    if (mutation == MUT_RES_NO_MEAN) singular_problem = 0;
    if (mutation == MUT_RES_MEAN_DIR) singular_problem = 1;
    double mean = singular_problem ? pairwise_sum(f, n) / (double)n : 0.0;
    double s2r = 0, s2f = 0, mr = 0, mf = 0;
    for (long t = 0; t < n; ++t) {
        double fb = f[t] - mean;
        double rv = fb - lp[t];
        if (r) r[t] = rv;
        s2r += rv * rv;
        s2f += fb * fb;
        if (fabs(rv) > mr) mr = fabs(rv);
        if (fabs(fb) > mf) mf = fabs(fb);
    }
    free(lp);
    if (rel_l2) {
        double q = (s2f > 0) ? s2r / s2f : s2r;
        *rel_l2 = (mutation == MUT_RES_NO_SQRT) ? q : sqrt(q);
    }
    if (rel_linf) *rel_linf = (mf > 0) ? mr / mf : mr;
    return 0;
}

int oracle_residual_bc(int nx, int ny, int nz, double dx, double dy, double dz, int bc_x,
                       int bc_y, int bc_z, const double *f, const double *p, double *r,
                       double *rel_l2, double *rel_linf)
{
    return oracle_residual_bc_mut(nx, ny, nz, dx, dy, dz, bc_x, bc_y, bc_z, f, p, r, rel_l2,
                                  rel_linf, MUT_NONE);
}

int oracle_residual(int nx, int ny, int nz, double dx, double dy, double dz, int bc_z,
                    const double *f, const double *p, double *r, double *rel_l2,
                    double *rel_linf)
{
    return oracle_residual_bc(nx, ny, nz, dx, dy, dz, ORC_PERIODIC, ORC_PERIODIC, bc_z, f, p, r,
                              rel_l2, rel_linf);
}

/*
 * The projection step around the solve (Section 3.3, the pressure equation
 * eqn:poisson and the velocity update eqn:corr; Section 3 for the
 * staggered layout).  Face velocities: u[k][j][i] sits on the east face of
 * cell (i,j,k), v on its north face, w on its top face.  Periodic directions
 * wrap; along an axis with walls (solid, no-slip: the pressure has zero
 * normal gradient there) the last face of the axis is the wall (u[nx-1],
 * v[ny-1] or w[nz-1] holds no flow and is not read) and no flux enters
 * through the first face either.
 *
 * oracle_divergence_bc: f = alpha * D u, the cell divergence
 *   (u[i] - u[i-1])/dx + (v[j] - v[j-1])/dy + (w[k] - w[k-1])/dz,
 * boundaries per axis: 0 periodic, 1 walls.
 */
/* flux through the faces below (lo) and above (hi) cell n of an axis of
 * N cells, faces holding face[n] (upper face of cell n) */
static void face_pair(const double *lo_face, const double *hi_face, int n, int N, int bc,
                      double *lo, double *hi)
{
    *lo = (n > 0) ? *lo_face : (bc == ORC_PERIODIC ? *lo_face : 0.0);
    *hi = (bc != ORC_PERIODIC && n == N - 1) ? 0.0 : *hi_face;
}

int oracle_divergence_bc(int nx, int ny, int nz, double dx, double dy, double dz, int bc_x,
                         int bc_y, int bc_z, const double *u, const double *v, const double *w,
                         double alpha, double *f)
{
    if (nx < 1 || ny < 1 || nz < 1 || !u || !v || !w || !f) return -1;
    if (bc_x < 0 || bc_x > 1 || bc_y < 0 || bc_y > 1 || bc_z < 0 || bc_z > 1) return -1;
#pragma omp parallel for schedule(static)
    for (long kk = 0; kk < (long)nz * ny; ++kk) {
        int k = (int)(kk / ny), j = (int)(kk % ny);
        int jm = (j + ny - 1) % ny, km = (k + nz - 1) % nz;
        for (int i = 0; i < nx; ++i) {
            int im = (i + nx - 1) % nx;
#define A(X, K, J, I) X[((long)(K) * ny + (J)) * nx + (I)]
            double ul, ur, vl, vr, wl, wr;
            face_pair(&A(u, k, j, im), &A(u, k, j, i), i, nx, bc_x, &ul, &ur);
            face_pair(&A(v, k, jm, i), &A(v, k, j, i), j, ny, bc_y, &vl, &vr);
            face_pair(&A(w, km, j, i), &A(w, k, j, i), k, nz, bc_z, &wl, &wr);
#undef A
            f[((long)k * ny + j) * nx + i] =
                alpha * ((ur - ul) / dx + (vr - vl) / dy + (wr - wl) / dz);
        }
    }
    return 0;
}

int oracle_divergence(int nx, int ny, int nz, double dx, double dy, double dz, int bc_z,
                      const double *u, const double *v, const double *w, double alpha,
                      double *f)
{
    return oracle_divergence_bc(nx, ny, nz, dx, dy, dz, ORC_PERIODIC, ORC_PERIODIC, bc_z, u, v,
                                w, alpha, f);
}

/*
 * oracle_correct_bc: u -= beta * G psi on every face, G the face gradient
 *   (psi[i+1] - psi[i])/dx on east faces, (psi[j+1] - psi[j])/dy on north
 *   faces, (psi[k+1] - psi[k])/dz on top faces; a wall face carries no
 *   gradient (zero normal pressure gradient), so u[nx-1], v[ny-1] or
 *   w[nz-1] of an axis with walls is left as it is.
 * With alpha * beta = 1 the corrected velocity is discretely divergence-free
 * whenever L psi = alpha D u, since D G = L (the 7-point operator with
 * mirrored ghosts at the walls).
 */
int oracle_correct_bc(int nx, int ny, int nz, double dx, double dy, double dz, int bc_x,
                      int bc_y, int bc_z, const double *psi, double beta, double *u, double *v,
                      double *w)
{
    if (nx < 1 || ny < 1 || nz < 1 || !psi || !u || !v || !w) return -1;
    if (bc_x < 0 || bc_x > 1 || bc_y < 0 || bc_y > 1 || bc_z < 0 || bc_z > 1) return -1;
#pragma omp parallel for schedule(static)
    for (long kk = 0; kk < (long)nz * ny; ++kk) {
        int k = (int)(kk / ny), j = (int)(kk % ny);
        int jp = (j + 1) % ny, kp = (k + 1) % nz;
        for (int i = 0; i < nx; ++i) {
            int ip = (i + 1) % nx;
            long c = ((long)k * ny + j) * nx + i;
#define P(K, J, I) psi[((long)(K) * ny + (J)) * nx + (I)]
            double pc = psi[c];
            if (!(bc_x != ORC_PERIODIC && i == nx - 1)) u[c] -= beta * (P(k, j, ip) - pc) / dx;
            if (!(bc_y != ORC_PERIODIC && j == ny - 1)) v[c] -= beta * (P(k, jp, i) - pc) / dy;
            if (!(bc_z != ORC_PERIODIC && k == nz - 1)) w[c] -= beta * (P(kp, j, i) - pc) / dz;
#undef P
        }
    }
    return 0;
}

int oracle_correct(int nx, int ny, int nz, double dx, double dy, double dz, int bc_z,
                   const double *psi, double beta, double *u, double *v, double *w)
{
    return oracle_correct_bc(nx, ny, nz, dx, dy, dz, ORC_PERIODIC, ORC_PERIODIC, bc_z, psi, beta,
                             u, v, w);
}

/*
 * Stretched z: walls in z and cell thicknesses h[0..nz-1] (nonuniform spacing
 * along z, uniform dx, dy).  Extends the z-direction elimination of Section
 * 3.3.1 to cells of different thickness; the paper's solver is described on
 * a uniform grid, so the operator here is the conservative (finite-volume)
 * reading of the same second-order stencil on the marker-and-cell grid:
 *
 *   (L_z p)_k = [ (p[k+1] - p[k]) / d[k+1/2] - (p[k] - p[k-1]) / d[k-1/2] ] / h[k],
 *   d[k+1/2] = (h[k] + h[k+1]) / 2   (distance between the cell centres),
 *
 * with no flux through a Neumann wall and, at a Dirichlet wall, the flux
 * (0 - p[0]) / (h[0]/2) to the zero value on the face (likewise at the top).
 * With equal thicknesses this is the uniform 7-point operator (the ghost
 * rules of the uniform case give the same wall rows).
 *
 * L is symmetric in the inner product weighted by the cell volumes, so the
 * singular (all-Neumann / periodic) problem is solvable for f with zero
 * volume-weighted mean: the solve removes mean_w(f) = sum h[k] f / sum h[k]
 * (over all cells) and returns the p with zero volume-weighted mean.
 */
static double mean_weighted(int nx, int ny, int nz, const double *h, const double *f,
                            int mutation)
{
    double num = 0.0, den = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double w = (mutation == MUT_H_MEAN) ? 1.0 : h[k];
        num += w * pairwise_sum(f + (long)k * nx * ny, (long)nx * ny);
        den += w * (double)nx * ny;
    }
    return num / den;
}

static double centre_distance(const double *h, int k, int mutation)
{
    /* between the centres of cells k and k+1 */
    return (mutation == MUT_H_FACE) ? h[k] : 0.5 * (h[k] + h[k + 1]);
}

/* One (mx,my) column: the rows of L_z + lam, multiplied by h[k] (symmetric
 * form), Gauss elimination without pivoting (Thomas).  Singular column: p[0]
 * pinned to 0, the first row dropped, the volume-weighted mean removed. */
static void zsolve_walls_h(int nz, const double *h, double lam, int singular,
                           double complex *g, double *lo, double *di, double *up, double *cp,
                           int bc_z, int mutation)
{
    for (int k = 0; k < nz; ++k) {
        lo[k] = (k > 0) ? 1.0 / centre_distance(h, k - 1, mutation) : 0.0;
        up[k] = (k < nz - 1) ? 1.0 / centre_distance(h, k, mutation) : 0.0;
        di[k] = lam * h[k] - lo[k] - up[k];
        if (bc_z == ORC_DIRICHLET) {
            if (k == 0) di[k] -= 2.0 / h[0];
            if (k == nz - 1) di[k] -= 2.0 / h[nz - 1];
        }
        g[k] *= h[k];
    }
    if (!singular) {
        thomas(nz, lo, di, up, g, cp);
        return;
    }
    if (nz == 1) { g[0] = 0.0; return; }
    thomas(nz - 1, lo + 1, di + 1, up + 1, g + 1, cp);
    g[0] = 0.0;
    double complex s = 0.0;
    double w = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double wk = (mutation == MUT_H_MEAN) ? 1.0 : h[k];
        s += wk * g[k];
        w += wk;
    }
    s /= w;
    for (int k = 0; k < nz; ++k) g[k] -= s;
}

/*
 * oracle_solve_bc_h: the solve on a z-stretched grid (bc_z Neumann or
 * Dirichlet walls; x and y as in oracle_solve_bc).  h: nz positive cell
 * thicknesses.  Singular problems (no Dirichlet axis): f minus its
 * volume-weighted mean (reported in rhs_mean), p with zero volume-weighted
 * mean.
 */
int oracle_solve_bc_h(int nx, int ny, int nz, double dx, double dy, const double *h, int bc_x,
                      int bc_y, int bc_z, const double *f, double *p, double *rhs_mean,
                      double *max_imag, int mutation)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0) || !(dy > 0) || !h || !f || !p) return -1;
    if (bc_x < 0 || bc_x > 2 || bc_y < 0 || bc_y > 2) return -1;
    if (bc_z != ORC_NEUMANN && bc_z != ORC_DIRICHLET) return -1;
    for (int k = 0; k < nz; ++k)
        if (!(h[k] > 0)) return -1;
    const int singular_problem =
        bc_x != ORC_DIRICHLET && bc_y != ORC_DIRICHLET && bc_z != ORC_DIRICHLET;
    long n = (long)nx * ny * nz, plane = (long)nx * ny;
    double complex *a = malloc(sizeof(double complex) * n);
    if (!a) return -1;

    double mean = singular_problem ? mean_weighted(nx, ny, nz, h, f, mutation) : 0.0;
    if (rhs_mean) *rhs_mean = mean;
    for (long t = 0; t < n; ++t) a[t] = f[t] - mean;

    if (bc_x == ORC_PERIODIC)
        dft_axis(a, nx, ny, nz, 0, -1, 1.0, mutation);
    else
        wall_axis(a, nx, ny, nz, 0, bc_x, 0, mutation);
    if (bc_y == ORC_PERIODIC)
        dft_axis(a, nx, ny, nz, 1, -1, 1.0, mutation);
    else
        wall_axis(a, nx, ny, nz, 1, bc_y, 0, mutation);

#pragma omp parallel
    {
        double complex *g = malloc(sizeof(double complex) * nz);
        double *lo = malloc(sizeof(double) * nz), *di = malloc(sizeof(double) * nz);
        double *up = malloc(sizeof(double) * nz), *cp = malloc(sizeof(double) * nz);
#pragma omp for schedule(static)
        for (long q = 0; q < plane; ++q) {
            int mx = (int)(q % nx), my = (int)(q / nx);
            double lam = eig_axis(bc_x, mx, nx, dx, mutation) + eig_axis(bc_y, my, ny, dy, mutation);
            int singular = singular_problem && mx == 0 && my == 0;
            for (int k = 0; k < nz; ++k) g[k] = a[(long)k * plane + q];
            zsolve_walls_h(nz, h, lam, singular, g, lo, di, up, cp, bc_z, mutation);
            for (int k = 0; k < nz; ++k) a[(long)k * plane + q] = g[k];
        }
        free(g); free(lo); free(di); free(up); free(cp);
    }

    if (bc_y == ORC_PERIODIC)
        dft_axis(a, nx, ny, nz, 1, +1, 1.0 / ny, mutation);
    else
        wall_axis(a, nx, ny, nz, 1, bc_y, 1, mutation);
    if (bc_x == ORC_PERIODIC)
        dft_axis(a, nx, ny, nz, 0, +1, 1.0 / nx, mutation);
    else
        wall_axis(a, nx, ny, nz, 0, bc_x, 1, mutation);

    double mre = 0.0, mim = 0.0;
    for (long t = 0; t < n; ++t) {
        p[t] = creal(a[t]);
        double re = fabs(creal(a[t])), im = fabs(cimag(a[t]));
        if (re > mre) mre = re;
        if (im > mim) mim = im;
    }
    if (max_imag) *max_imag = (mre > 0) ? mim / mre : mim;
    free(a);
    if (singular_problem) {
        double pm = mean_weighted(nx, ny, nz, h, p, mutation);
        for (long t = 0; t < n; ++t) p[t] -= pm;
    }
    return 0;
}

/* out = L p on the z-stretched grid (x and y as in oracle_laplacian_bc) */
int oracle_laplacian_bc_h(int nx, int ny, int nz, double dx, double dy, const double *h,
                          int bc_x, int bc_y, int bc_z, const double *p, double *out,
                          int mutation)
{
    if (nx < 1 || ny < 1 || nz < 1 || !h || !p || !out) return -1;
    if (bc_z != ORC_NEUMANN && bc_z != ORC_DIRICHLET) return -1;
    double ax = 1.0 / (dx * dx), ay = 1.0 / (dy * dy);
#pragma omp parallel for schedule(static)
    for (long kk = 0; kk < (long)nz * ny; ++kk) {
        int k = (int)(kk / ny), j = (int)(kk % ny);
        double fjm, fjp;
        int jm = nbr(j, -1, ny, bc_y, &fjm), jp = nbr(j, +1, ny, bc_y, &fjp);
        for (int i = 0; i < nx; ++i) {
            double fim, fip;
            int im = nbr(i, -1, nx, bc_x, &fim), ip = nbr(i, +1, nx, bc_x, &fip);
#define P(K, J, I) p[((long)(K) * ny + (J)) * nx + (I)]
            double c = P(k, j, i);
            double flux_up = 0.0, flux_dn = 0.0; /* through the top and bottom faces */
            if (k < nz - 1)
                flux_up = (P(k + 1, j, i) - c) / centre_distance(h, k, mutation);
            else if (bc_z == ORC_DIRICHLET)
                flux_up = (0.0 - c) / (0.5 * h[k]);
            if (k > 0)
                flux_dn = (c - P(k - 1, j, i)) / centre_distance(h, k - 1, mutation);
            else if (bc_z == ORC_DIRICHLET)
                flux_dn = (c - 0.0) / (0.5 * h[k]);
            double v = ax * (fip * P(k, j, ip) - 2.0 * c + fim * P(k, j, im)) +
                       ay * (fjp * P(k, jp, i) - 2.0 * c + fjm * P(k, jm, i)) +
                       (flux_up - flux_dn) / h[k];
#undef P
            out[((long)k * ny + j) * nx + i] = v;
        }
    }
    return 0;
}

/* r = (f - mean_w(f)) - L p on the z-stretched grid (the weighted mean
 * removed only when no axis is Dirichlet), relative L2 and Linf norms */
int oracle_residual_bc_h(int nx, int ny, int nz, double dx, double dy, const double *h,
                         int bc_x, int bc_y, int bc_z, const double *f, const double *p,
                         double *r, double *rel_l2, double *rel_linf, int mutation)
{
    long n = (long)nx * ny * nz;
    double *lp = malloc(sizeof(double) * n);
    if (!lp) return -1;
    if (oracle_laplacian_bc_h(nx, ny, nz, dx, dy, h, bc_x, bc_y, bc_z, p, lp, mutation)) {
        free(lp);
        return -1;
    }
    int singular_problem =
        bc_x != ORC_DIRICHLET && bc_y != ORC_DIRICHLET && bc_z != ORC_DIRICHLET;
    double mean = singular_problem ? mean_weighted(nx, ny, nz, h, f, mutation) : 0.0;
    double s2r = 0, s2f = 0, mr = 0, mf = 0;
    for (long t = 0; t < n; ++t) {
        double fb = f[t] - mean;
        double rv = fb - lp[t];
        if (r) r[t] = rv;
        s2r += rv * rv;
        s2f += fb * fb;
        if (fabs(rv) > mr) mr = fabs(rv);
        if (fabs(fb) > mf) mf = fabs(fb);
    }
    free(lp);
    if (rel_l2) *rel_l2 = (s2f > 0) ? sqrt(s2r / s2f) : sqrt(s2r);
    if (rel_linf) *rel_linf = (mf > 0) ? mr / mf : mr;
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
