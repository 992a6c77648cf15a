// k_zperiodic.hip -- z solve for triply periodic boxes: the eigen-expansion
// of FluTAS Section 3.3.1 applied along z as well.  For each column (m, ky)
// of the spectrum one workgroup-resident pass does
//     forward FFT along z -> multiply by 1/((lam_x + lam_y + lam_z) nx ny nz)
//     (the (0,0,0) mode, the mean, is set to zero) -> inverse FFT along z,
// reading and writing HBM once.  lam(j) = -(4/h^2) sin^2(pi j/n).
//
// Column m = 0 packs the DC and Nyquist x-modes as A + iB (see k_xpass.hip);
// after the y and z transforms they separate through the Hermitian symmetry
// of each real mode in (ky, kz):
//     A(ky,kz) = (Z(ky,kz) + conj Z(-ky,-kz))/2,
//     B(ky,kz) = (Z(ky,kz) - conj Z(-ky,-kz))/(2i).
// The first `nspecial` workgroups take the column pairs (ky, -ky) of m = 0,
// scale A and B with their own eigenvalues and recombine.
#include "fft_core.hpp"
#include "lengths.hpp"

#ifndef PK_REAL
#error "PK_REAL must be defined"
#endif

namespace pk {
namespace PK_NS {

using R = PK_REAL;

#include "zper_body.hpp"

template <int N>
__global__ __launch_bounds__(ZPCfg<N>::NT) void k_z_per(ZArgs a0, int nspecial)
{
    using B = ZPBody<N>;
    __shared__ __align__(16) char s_lds[B::LDS_BYTES];
    B::run(a0, VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x}, nspecial, s_lds);
}

template <int N> static int run_zp(const ZArgs &a, hipStream_t s)
{
    using Cf = ZPCfg<N>;
    const int npairs = a.ny / 2 + 1;
    constexpr int NB = Cf::NB, NP = Cf::NB / 2;
    int nspecial, nmain = (a.ny * a.M + NB - 1) / NB;
    if (a.xwall) {
        nspecial = a.ywall ? a.ny * ((a.M + NB - 1) / NB) : npairs * ((a.M + NP - 1) / NP);
        nmain = 0;
    } else {
        nspecial = a.ywall ? (a.ny + NB - 1) / NB : (npairs + NP - 1) / NP;
    }
    hipLaunchKernelGGL(k_z_per<N>, dim3(nspecial + nmain, a.batch ? a.nbatch : 1), dim3(Cf::NT),
                       0, s, a, nspecial);
    return (int)hipGetLastError();
}

}  // namespace PK_NS
using namespace PK_NS;

#define PK_CASE_ZP(N) case N: return run_zp<N>(a, s);

int PK_SUFFIX(launch_z_periodic)(const ZArgs &a, hipStream_t s)
{
    switch (a.nz) { PK_LENGTHS(PK_CASE_ZP) default: return -1; }
}

}  // namespace pk
