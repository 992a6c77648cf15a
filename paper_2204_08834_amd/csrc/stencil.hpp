// stencil.hpp -- the nearest-neighbour stencils of the marker-and-cell grid
// (FluTAS Sections 3 and 3.3), in FP64: the residual of the discrete Poisson
// equation, r = (f - mean f) - L p, with L the 7-point operator of Section
// 3.3.1 (periodic in x and y; in z periodic, or with the mirrored ghost value
// at the walls: zero normal gradient on the wall face); the divergence of the
// face velocities (the right-hand side of the projection step); and the
// velocity correction with the pressure update.
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
// default), halved (down to 1) while the nb problems of a batched launch
// would get fewer than 1024 workgroups together, so that small grids still
// fill the device.  nb is the size of the problem group, not the number of
// problems a launch still serves, so that every launch of the group tiles
// and sums the same way.  Each range re-reads two planes of p, so deeper
// ranges read less.  A negative kr_max is an exact depth (-kr_max planes,
// no halving): the plan picks it so that the workgroups fill the resident
// slots of the device in whole rounds.
__host__ __device__ constexpr int march_planes(int ny, int nz, int tj, int kr_max, int nb = 1)
{
    if (kr_max < 0) return -kr_max < nz ? -kr_max : (nz > 0 ? nz : 1);
    int kr = kr_max > 0 ? kr_max : 8;
    const int b = nb > 1 ? nb : 1;
    while (kr > 1 && march_jblocks(ny, tj) * ((nz + kr - 1) / kr) * b < 1024) kr /= 2;
    return kr;
}
__host__ __device__ constexpr int march_kblocks(int ny, int nz, int tj, int kr_max, int nb = 1)
{
    const int kr = march_planes(ny, nz, tj, kr_max, nb);
    return (nz + kr - 1) / kr;
}

// Indexing of a plane tile: TJ consecutive y-rows (all of x) of one z-plane,
// M pairs (2h, 2h+1) per row, spread over the NT threads of a workgroup.
template <int M, int TJ, int NT>
struct MarchIdx {
    static constexpr int NX = 2 * M;
    static constexpr int E = TJ * M;  // pairs per plane tile
    static constexpr int PER = (E + NT - 1) / NT;
    static constexpr bool EXACT = (E % NT) == 0;

    int ny, nz, bc_z, bc_x = 0;
    int j0, V;     // first y-row and number of valid rows of this block
    int jm, jn;    // halo rows: (j0 - 1) mod ny and (j0 + V) mod ny, or the wall row
    double sm, sn; // factors of the halo rows: -1 for the ghost of a Dirichlet wall
    size_t plane;  // ny * NX

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

    // bc: 0 periodic, 1 Neumann walls (the ghost row mirrors the wall row),
    // 2 Dirichlet walls (the ghost row is the negated wall row)
    __device__ __forceinline__ void setup(int jb, int ny_, int nz_, int bc_z_, int bc_y = 0)
    {
        ny = ny_;
        nz = nz_;
        bc_z = bc_z_;
        j0 = jb * TJ;
        V = ny - j0 < TJ ? ny - j0 : TJ;
        const bool lo = j0 == 0, hi = j0 + V == ny;
        jm = lo ? (bc_y == 0 ? ny - 1 : 0) : j0 - 1;
        jn = hi ? (bc_y == 0 ? 0 : ny - 1) : j0 + V;
        sm = (lo && bc_y == 2) ? -1.0 : 1.0;
        sn = (hi && bc_y == 2) ? -1.0 : 1.0;
        plane = (size_t)ny * NX;
    }
};

// a pair of p as stored (FP64, or FP32 for the first iterate) and its exact
// FP64 value
template <class T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };
__device__ __forceinline__ double2 widen(double2 v) { return v; }
__device__ __forceinline__ double2 widen(float2 v) { return double2{(double)v.x, (double)v.y}; }

template <int M, int TJ, int NT, class PT = double>
struct PlaneMarch : MarchIdx<M, TJ, NT> {
    using B = MarchIdx<M, TJ, NT>;
    using B::PER;
    using B::NX;
    using B::plane;
    using B::roff;
    using B::valid;
    using B::row_of;
    using B::pair_of;
    using B::kdown;
    using B::kup;
    using B::jm;
    using B::jn;
    using B::V;

    const PK_GLOBAL double *f;  // set through gbl()
    const PK_GLOBAL PT *p;
    double ax, ay, az, mu;
    const double *zc = nullptr;  // stretched z: per-plane coefficients (XFwdArgs::zc)
    double2 (*tile)[M];  // LDS, TJ + 2 rows

    // p is held as loaded (FP32 pairs for the refinement's first iterate,
    // widened exactly where used): planes k-1 and k, and the inputs of step
    // k that fetch(k) loads -- p at plane k+1, f at plane k and the two halo
    // rows of plane k.
    using P2 = typename Pair<PT>::type;
    static constexpr int HPER = (M + NT - 1) / NT;  // halo pairs per thread
    P2 pd[PER], pc[PER];
    P2 pun[PER], hmn[HPER], hnn[HPER];
    double2 fvn[PER];

    // p at planes k0-1 and k0 into registers.  Elements past the last row
    // of the grid load from the start of the plane (in bounds, never used):
    // branch-free loads.
    __device__ __forceinline__ void start(int k0)
    {
        const PK_GLOBAL PT *pdn = p + (size_t)kdown(k0) * plane;
        const PK_GLOBAL PT *pcn = p + (size_t)k0 * plane;
        // below a Dirichlet bottom wall the ghost plane is -p(0)
        const PT gs = (k0 == 0 && this->bc_z == 2) ? PT(-1) : PT(1);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = roff(q);
            const P2 x = *(const PK_GLOBAL P2 *)(pdn + o);
            pd[q] = P2{gs * x.x, gs * x.y};
            pc[q] = *(const PK_GLOBAL P2 *)(pcn + o);
        }
    }

    // The loads of step k (the halo rows of plane k, p at plane k+1, f at
    // plane k); halo lanes past the row load pair 0 (in bounds, never used).
    // The halo rows go first: loads complete in issue order, so the wait for
    // the halo rows (staged in LDS before the barrier of step k) leaves the
    // other loads in flight across that barrier.  Issued last, the halo
    // loads made the check 5 % slower on MI355X.
    __device__ __forceinline__ void fetch(int k)
    {
        const PK_GLOBAL PT *pup = p + (size_t)kup(k) * plane;
        const PK_GLOBAL double *fk = f + (size_t)k * plane;
        const PK_GLOBAL PT *pk_ = p + (size_t)k * plane;
#pragma unroll
        for (int i = 0; i < HPER; ++i) {
            const int h = threadIdx.x + i * NT;
            const int hc = (M % NT == 0 || h < M) ? h : 0;
            hmn[i] = *(const PK_GLOBAL P2 *)(pk_ + (size_t)jm * NX + 2 * hc);
            hnn[i] = *(const PK_GLOBAL P2 *)(pk_ + (size_t)jn * NX + 2 * hc);
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = roff(q);
            pun[q] = *(const PK_GLOBAL P2 *)(pup + o);
            fvn[q] = *(const PK_GLOBAL double2 *)(fk + o);
        }
    }

    // Residual at plane k from the inputs fetch(k) loaded: sink(q, t, h, r0,
    // r1, f0, f1, pc) for every valid element (row j0 + t, pair h).  The
    // caller syncs before the next step (the LDS tile is rewritten).
    template <class Sink>
    __device__ __forceinline__ void step(int k, Sink &sink)
    {
        // above a Dirichlet top wall the ghost plane is -p(nz-1)
        const PT gs = (k == this->nz - 1 && this->bc_z == 2) ? PT(-1) : PT(1);
        const double sm = this->sm, sn = this->sn;
        // stretched z: the fluxes through the faces below and above
        const bool zs = zc != nullptr;
        const double czm = zs ? zc[2 * k] : 0.0, czp = zs ? zc[2 * k + 1] : 0.0;
#pragma unroll
        for (int i = 0; i < HPER; ++i) {
            const int h = threadIdx.x + i * NT;
            if (M % NT == 0 || h < M) {
                const double2 a = widen(hmn[i]), b = widen(hnn[i]);
                tile[0][h] = double2{sm * a.x, sm * a.y};
                tile[V + 1][h] = double2{sn * b.x, sn * b.y};
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (valid(q)) tile[row_of(q) + 1][pair_of(q)] = widen(pc[q]);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            pun[q] = P2{gs * pun[q].x, gs * pun[q].y};
            if (valid(q)) {
                const int t = row_of(q), h = pair_of(q);
                const double2 ps = tile[t][h], pn = tile[t + 2][h];
                const double2 c = widen(pc[q]), d = widen(pd[q]), u = widen(pun[q]);
                // x neighbours; at walls along x the ghost is the wall cell
                // (Neumann) or its negation (Dirichlet)
                const int bx = this->bc_x;
                const double pl = h != 0 ? tile[t + 1][h - 1].y
                                         : (bx == 0 ? tile[t + 1][M - 1].y : (bx == 1 ? c.x : -c.x));
                const double pq = h != M - 1 ? tile[t + 1][h + 1].x
                                             : (bx == 0 ? tile[t + 1][0].x : (bx == 1 ? c.y : -c.y));
                const double z0 = zs ? czp * (u.x - c.x) - czm * (c.x - d.x)
                                     : az * (u.x - 2.0 * c.x + d.x);
                const double z1 = zs ? czp * (u.y - c.y) - czm * (c.y - d.y)
                                     : az * (u.y - 2.0 * c.y + d.y);
                const double l0 = ax * (c.y - 2.0 * c.x + pl) + ay * (pn.x - 2.0 * c.x + ps.x) + z0;
                const double l1 = ax * (pq - 2.0 * c.y + c.x) + ay * (pn.y - 2.0 * c.y + ps.y) + z1;
                const double f0 = fvn[q].x - mu, f1 = fvn[q].y - mu;
                sink(q, t, h, f0 - l0, f1 - l1, f0, f1, c);
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            pd[q] = pc[q];
            pc[q] = pun[q];
        }
    }
};

// Cell-centred divergence of face velocities on the marker-and-cell grid
// (FluTAS Section 3, right-hand side of eqn:poisson):
//   f = cx (u_i - u_{i-1}) + cy (v_j - v_{j-1}) + cz (w_k - w_{k-1}),
// cx = alpha/dx etc., with u on east faces, v on north faces and w on top
// faces of the cells; x and y periodic; in z periodic, or walls with no flux
// through the bottom face of plane 0 and the top face of plane nz-1 (the
// value stored there is not read).  Same 2.5-D march as the residual: w of
// plane k-1 is kept in registers, the v rows of plane k with the halo row
// j0-1 and the odd u value of every pair are staged in LDS for the y and x
// neighbours.  Reads per output row: u, v, w and 1/TJ halo rows.
template <int M, int TJ, int NT>
struct DivMarch : MarchIdx<M, TJ, NT> {
    using B = MarchIdx<M, TJ, NT>;
    using B::PER;
    using B::plane;
    using B::roff;
    using B::valid;
    using B::row_of;
    using B::pair_of;
    using B::jm;

    const PK_GLOBAL double *u, *v, *w;  // set through gbl()
    double cx, cy, cz;
    bool xwall = false, ywall = false;  // solid walls along x / y: no flux through
                                        // the first face or the last (wall) face
    double2 (*vt)[M];  // LDS: TJ + 1 rows (row 0: the halo row j0 - 1)
    double (*ut)[M];   // LDS: TJ rows of u[2h+1]
    double2 wd[PER];   // w of plane k-1 (the flux through the bottom face)

    // LDS bytes of the two staging arrays
    static constexpr size_t lds_bytes() { return sizeof(double2) * (TJ + 1) * M + sizeof(double) * TJ * M; }
    __device__ __forceinline__ void bind(char *lds)
    {
        vt = (double2(*)[M])lds;
        ut = (double(*)[M])(lds + sizeof(double2) * (TJ + 1) * M);
    }

    __device__ __forceinline__ void start(int k0)
    {
        const bool none = k0 == 0 && this->bc_z != 0;  // bottom wall
        const PK_GLOBAL double *wdn = w + (size_t)B::kdown(k0) * plane;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const double2 x = *(const PK_GLOBAL double2 *)(wdn + roff(q));
            wd[q] = none ? double2{0.0, 0.0} : x;
        }
    }

    // sink(q, t, h, f0, f1) for every valid element (row j0 + t, pair h);
    // the caller syncs before the next step (the LDS arrays are rewritten)
    template <class Sink>
    __device__ __forceinline__ void step(int k, Sink &sink)
    {
        const size_t kp = (size_t)k * plane;
        double2 uu[PER], vv[PER], ww[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = roff(q);
            uu[q] = ld_stream(u + kp + o);
            vv[q] = *(const PK_GLOBAL double2 *)(v + kp + o);  // also a halo row
            ww[q] = *(const PK_GLOBAL double2 *)(w + kp + o);  // also read at k + 1
        }
        const bool vnone = ywall && this->j0 == 0;  // no flux below row 0
        for (int h = threadIdx.x; h < M; h += NT) {
            const double2 x = *(const PK_GLOBAL double2 *)(v + kp + (size_t)jm * B::NX + 2 * h);
            vt[0][h] = vnone ? double2{0.0, 0.0} : x;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (valid(q)) {
                vt[row_of(q) + 1][pair_of(q)] = vv[q];
                ut[row_of(q)][pair_of(q)] = uu[q].y;
            }
        __syncthreads();
        const bool top = k == this->nz - 1 && this->bc_z != 0;  // top wall
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (valid(q)) {
                const int t = row_of(q), h = pair_of(q);
                const double ul = (xwall && h == 0) ? 0.0 : ut[t][h == 0 ? M - 1 : h - 1];
                const double ur = (xwall && h == M - 1) ? 0.0 : uu[q].y;  // the wall face
                const double2 vs = vt[t][h];
                const double2 vn = (ywall && this->j0 + t == this->ny - 1) ? double2{0.0, 0.0}
                                                                           : vv[q];
                const double2 wu = top ? double2{0.0, 0.0} : ww[q];
                const double f0 = cx * (uu[q].x - ul) + cy * (vn.x - vs.x) + cz * (wu.x - wd[q].x);
                const double f1 = cx * (ur - uu[q].x) + cy * (vn.y - vs.y) + cz * (wu.y - wd[q].y);
                sink(q, t, h, f0, f1);
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) wd[q] = ww[q];
    }
};

// Velocity correction and pressure update of the projection step (FluTAS
// Section 3.3, eqn:corr and eqn:p_upt) from the solution psi:
//   u -= bx (psi_{i+1} - psi_i),  v -= by (psi_{j+1} - psi_j),
//   w -= bz (psi_{k+1} - psi_k),  p += psi,
// bx = beta/dx etc., on the faces of the divergence above: x and y periodic;
// in z periodic, or walls, where w on the top face of plane nz-1 (the wall)
// is left as it is.  psi of plane k+1 is read once per plane into registers
// and kept as the next plane's centre; the plane-k tile and the halo row
// j0+V are staged in LDS for the x and y neighbours.
template <int M, int TJ, int NT>
struct CorrMarch : MarchIdx<M, TJ, NT> {
    using B = MarchIdx<M, TJ, NT>;
    using B::PER;
    using B::plane;
    using B::roff;
    using B::valid;
    using B::row_of;
    using B::pair_of;
    using B::jn;
    using B::V;

    const PK_GLOBAL double *psi;
    PK_GLOBAL double *u, *v, *w, *p;  // p may be null
    double bx, by, bz;
    bool xwall = false, ywall = false;  // wall faces (u[nx-1], v[ny-1]) stay as they are
    double2 (*tile)[M];  // LDS: TJ + 1 rows (row V: the halo row j0 + V)
    double2 pc[PER];     // psi of plane k

    static constexpr size_t lds_bytes() { return sizeof(double2) * (TJ + 1) * M; }

    __device__ __forceinline__ void start(int k0)
    {
        const PK_GLOBAL double *c = psi + (size_t)k0 * plane;
#pragma unroll
        for (int q = 0; q < PER; ++q) pc[q] = *(const PK_GLOBAL double2 *)(c + roff(q));
    }

    // the caller syncs before the next step (the LDS tile is rewritten)
    __device__ __forceinline__ void step(int k)
    {
        const size_t kp = (size_t)k * plane;
        const PK_GLOBAL double *pup = psi + (size_t)B::kup(k) * plane;
        const bool top = k == this->nz - 1 && this->bc_z != 0;  // top wall: w stays
        double2 pu[PER], uu[PER], vv[PER], ww[PER], pp[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = roff(q);
            pu[q] = *(const PK_GLOBAL double2 *)(pup + o);
            uu[q] = ld_stream(u + kp + o);
            vv[q] = ld_stream(v + kp + o);
            ww[q] = ld_stream(w + kp + o);
            if (p) pp[q] = ld_stream(p + kp + o);
        }
        for (int h = threadIdx.x; h < M; h += NT)
            tile[V][h] = *(const PK_GLOBAL double2 *)(psi + kp + (size_t)jn * B::NX + 2 * h);
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (valid(q)) tile[row_of(q)][pair_of(q)] = pc[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (valid(q)) {
                const int t = row_of(q), h = pair_of(q), o = roff(q);
                const double2 c = pc[q];
                const double pr = tile[t][h == M - 1 ? 0 : h + 1].x;  // psi_{2h+2}
                const double2 pn = tile[t + 1][h];                     // psi of row j + 1
                double2 a = uu[q], b = vv[q];
                a.x -= bx * (c.y - c.x);
                if (!(xwall && h == M - 1)) a.y -= bx * (pr - c.y);
                if (!(ywall && this->j0 + t == this->ny - 1)) {
                    b.x -= by * (pn.x - c.x);
                    b.y -= by * (pn.y - c.y);
                }
                st_stream(u + kp + o, a);
                st_stream(v + kp + o, b);
                if (!top) {
                    double2 d = ww[q];
                    d.x -= bz * (pu[q].x - c.x);
                    d.y -= bz * (pu[q].y - c.y);
                    st_stream(w + kp + o, d);
                }
                if (p) {
                    double2 e = pp[q];
                    e.x += c.x;
                    e.y += c.y;
                    st_stream(p + kp + o, e);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) pc[q] = pu[q];
    }
};

// sum three doubles over the workgroup; thread 0 gets the totals (the
// caller's `sh` holds 3 doubles per wavefront; the call syncs)
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *sh,
                                           int nthreads = 0)
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
        const int nw = ((nthreads > 0 ? nthreads : (int)blockDim.x) + 63) >> 6;
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
