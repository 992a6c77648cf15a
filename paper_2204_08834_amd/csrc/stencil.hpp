// stencil.hpp -- FP64 residual of the discrete Poisson equation on the
// marker-and-cell grid, r = (f - mean f) - L p, with L the 7-point operator
// of FluTAS Section 3.3.1: periodic in x and y; in z periodic, or with the
// mirrored ghost value at the walls (zero normal gradient on the wall face).
//
// 2.5-D blocking.  A workgroup owns TJ consecutive y-rows (all of x) and
// marches up a range of z-planes.  Each thread keeps p at planes k-1, k, k+1
// of its points in registers, so every p value is read from memory once per
// plane range; the plane-k tile plus one halo row on each side in y is staged
// in LDS, from which the x and y neighbours are taken.  Reads per output row:
// f, p(k+1) and 2/TJ halo rows, against seven row-reads for a plain stencil.
// Points are handled in pairs (2h, 2h+1) as double2.
#pragma once
#include "common.hpp"

namespace pk {

// rows per workgroup for rows of M pairs: about `pairs` pairs per plane
// tile.  The residual check streams best with 2048 pairs; the residual pass
// with transform, which also holds an FFT tile, with 1024 (more workgroups,
// fewer registers): measured on MI355X at 512x512x256 and 256^3.
constexpr int march_rows(int M, int pairs = 2048)
{
    const int t = pairs / M;
    return t < 1 ? 1 : (t > 16 ? 16 : t);
}
constexpr int march_rows_res(int M) { return march_rows(M, 1024); }
// workgroups of one problem: (y-row blocks) x (z-plane ranges), plane-major
__host__ __device__ constexpr int march_jblocks(int ny, int tj) { return (ny + tj - 1) / tj; }

// z-planes per workgroup: kr_max (8 by default, a tuning knob; 0 means the
// default), halved (down to 1) while a problem would get fewer than 1024
// workgroups, so that small grids still fill the device.  Each range
// re-reads two planes of p, so deeper ranges read less.
__host__ __device__ constexpr int march_planes(int ny, int nz, int tj, int kr_max)
{
    int kr = kr_max > 0 ? kr_max : 8;
    while (kr > 1 && march_jblocks(ny, tj) * ((nz + kr - 1) / kr) < 1024) kr /= 2;
    return kr;
}
__host__ __device__ constexpr int march_kblocks(int ny, int nz, int tj, int kr_max)
{
    const int kr = march_planes(ny, nz, tj, kr_max);
    return (nz + kr - 1) / kr;
}

template <int M, int TJ, int NT>
struct PlaneMarch {
    static constexpr int NX = 2 * M;
    static constexpr int E = TJ * M;  // pairs per plane tile
    static constexpr int PER = (E + NT - 1) / NT;
    static constexpr bool EXACT = (E % NT) == 0;

    const PK_GLOBAL double *f, *p;  // set through gbl()
    int ny, nz, bc_z;
    double ax, ay, az, mu;
    int j0, V;     // first y-row and number of valid rows of this block
    int jm, jn;    // halo rows: (j0 - 1) mod ny and (j0 + V) mod ny
    size_t plane;  // ny * NX
    double2 (*tile)[M];  // LDS, TJ + 2 rows
    double2 pd[PER], pc[PER];

    // Element q of a thread is (row t, pair h) with e = threadIdx.x + q NT,
    // t = e / M, h = e % M.  When NT divides M (ROWSPLIT) the row of element q
    // is the same for the whole workgroup (t = q / (M/NT)), so the row offset
    // is a uniform value and only the pair offset varies per lane.
    static constexpr bool ROWSPLIT = (M % NT) == 0;
    static constexpr int SPR = ROWSPLIT ? M / NT : 1;  // elements per row and thread

    __device__ __forceinline__ int elem(int q) const { return threadIdx.x + q * NT; }
    __device__ __forceinline__ int row_of(int q) const
    {
        return ROWSPLIT ? q / SPR : elem(q) / M;
    }
    __device__ __forceinline__ int pair_of(int q) const
    {
        return ROWSPLIT ? (int)threadIdx.x + (q % SPR) * NT : elem(q) - (elem(q) / M) * M;
    }
    __device__ __forceinline__ bool valid(int q) const
    {
        if constexpr (ROWSPLIT) return q / SPR < V;
        const int e = elem(q);
        return (EXACT || e < E) && e / M < V;
    }
    // offset of element q within a plane; rows past the grid are clamped to
    // the first row of the block (loaded, never used): branch-free loads
    __device__ __forceinline__ int roff(int q) const
    {
        if constexpr (ROWSPLIT) {
            const int t = q / SPR < V ? q / SPR : 0;
            return (j0 + t) * NX + 2 * pair_of(q);
        }
        const int e = elem(q), t = e / M, h = e - t * M;
        return valid(q) ? (j0 + t) * NX + 2 * h : 0;
    }
    __device__ __forceinline__ int kdown(int k) const
    {
        return k > 0 ? k - 1 : (bc_z == 0 ? nz - 1 : 0);
    }
    __device__ __forceinline__ int kup(int k) const
    {
        return k < nz - 1 ? k + 1 : (bc_z == 0 ? 0 : k);
    }

    __device__ __forceinline__ void setup(int jb, int ny_, int nz_, int bc_z_)
    {
        ny = ny_;
        nz = nz_;
        bc_z = bc_z_;
        j0 = jb * TJ;
        V = ny - j0 < TJ ? ny - j0 : TJ;
        jm = j0 == 0 ? ny - 1 : j0 - 1;
        jn = j0 + V == ny ? 0 : j0 + V;
        plane = (size_t)ny * NX;
    }

    // p at planes k0-1 and k0 into registers.  Elements past the last row
    // of the grid load from the start of the plane (in bounds, never used):
    // branch-free loads.
    __device__ __forceinline__ void start(int k0)
    {
        const PK_GLOBAL double *pdn = p + (size_t)kdown(k0) * plane;
        const PK_GLOBAL double *pcn = p + (size_t)k0 * plane;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = roff(q);
            pd[q] = *(const PK_GLOBAL double2 *)(pdn + o);
            pc[q] = *(const PK_GLOBAL double2 *)(pcn + o);
        }
    }

    // Residual at plane k: sink(q, t, h, r0, r1, f0, f1, pc) for every valid
    // element (row j0 + t, pair h).  The caller syncs before the next step
    // (the LDS tile is rewritten).
    template <class Sink>
    __device__ __forceinline__ void step(int k, Sink &sink)
    {
        const PK_GLOBAL double *pup = p + (size_t)kup(k) * plane;
        const PK_GLOBAL double *fk = f + (size_t)k * plane;
        const PK_GLOBAL double *pk_ = p + (size_t)k * plane;
        double2 pu[PER], fv[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = roff(q);
            pu[q] = *(const PK_GLOBAL double2 *)(pup + o);
            fv[q] = *(const PK_GLOBAL double2 *)(fk + o);
        }
        for (int h = threadIdx.x; h < M; h += NT) {
            tile[0][h] = *(const PK_GLOBAL double2 *)(pk_ + (size_t)jm * NX + 2 * h);
            tile[V + 1][h] = *(const PK_GLOBAL double2 *)(pk_ + (size_t)jn * NX + 2 * h);
        }
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (valid(q)) tile[row_of(q) + 1][pair_of(q)] = pc[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (valid(q)) {
                const int t = row_of(q), h = pair_of(q);
                const double2 ps = tile[t][h], pn = tile[t + 2][h];
                const double pl = tile[t + 1][h == 0 ? M - 1 : h - 1].y;
                const double pq = tile[t + 1][h == M - 1 ? 0 : h + 1].x;
                const double2 c = pc[q], d = pd[q], u = pu[q];
                const double l0 = ax * (c.y - 2.0 * c.x + pl) + ay * (pn.x - 2.0 * c.x + ps.x) +
                                  az * (u.x - 2.0 * c.x + d.x);
                const double l1 = ax * (pq - 2.0 * c.y + c.x) + ay * (pn.y - 2.0 * c.y + ps.y) +
                                  az * (u.y - 2.0 * c.y + d.y);
                const double f0 = fv[q].x - mu, f1 = fv[q].y - mu;
                sink(q, t, h, f0 - l0, f1 - l1, f0, f1, c);
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            pd[q] = pc[q];
            pc[q] = pu[q];
        }
    }
};

// sum three doubles over the workgroup; thread 0 gets the totals (the
// caller's `sh` holds 3 doubles per wavefront; the call syncs)
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
        c += __shfl_down(c, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sh[3 * wid] = a;
        sh[3 * wid + 1] = b;
        sh[3 * wid + 2] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        a = 0.0;
        b = 0.0;
        c = 0.0;
        for (int w = 0; w < nw; ++w) {
            a += sh[3 * w];
            b += sh[3 * w + 1];
            c += sh[3 * w + 2];
        }
    }
}

}  // namespace pk
