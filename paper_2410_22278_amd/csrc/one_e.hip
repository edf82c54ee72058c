// Gamma-point one-electron terms: overlap S, kinetic T, nuclear attraction V
// and the nuclear repulsion energy E_nuc, on the pair list, lattice and
// reciprocal vectors of the J/K build.
//
// Per unique local primitive pair (one thread per (shell pair, image) group):
//   S += cpre (pi/p)^{3/2} E^{ix jx}_0 E^{iy jy}_0 E^{iz jz}_0              (Sec. 2.2, eq. pbc_overlap_formula)
//   T += cpre (pi/p)^{3/2} sum_x [-jx(jx-1)/2 E^{i,j-2}_0 + (2jx+1) b E^{i,j}_0
//                                   - 2 b^2 E^{i,j+2}_0] E_0(y) E_0(z)       (supporting information, eq. kinetic_formula)
//   V += q_C cpre (2 pi/p) sum_{R_C} sum_t E^{ab}_t R^SR_t(p, P - C - R_C)  (Sec. 2.3, eq. pbc_v1e_general_final)
// into halves X (M = X + X^T, the pair symmetry weights being in cpre), with
// the short-range point-charge kernel erfc(w r)/r, R_C inside the sphere of
// eq. pbc_v1e_real_cutoff_implementation.  The reciprocal part of V uses the
// pair structure factors of the reciprocal exchange with the nuclear
// structure factor rho_n(G) = sum_C q_C e^{-i G.C} in place of the density's;
// the self term is -(pi/(V w^2)) sum_C q_C S.  E_nuc is the Ewald energy of
// the point charges (Sec. 2.9, eq. nuclear_repulsion_energy).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.h"
#include "kernels.h"

namespace pbcjk {

namespace {

template <int LA, int LB>
__global__ __launch_bounds__(256) void k_one_e(OneEArgs a)
{
    constexpr int L = LA + LB;
    constexpr int NA = ncart(LA), NB = ncart(LB);
    __shared__ double tab[kBoysNT * kBoysTerms];
    __shared__ double etab[kBoysNT];
    constexpr double kInvFact[kBoysTerms] = {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720,
                                             1.0 / 5040, 1.0 / 40320};
    for (int i = threadIdx.x; i < kBoysNT * kBoysTerms; i += blockDim.x) {
        int k = i / kBoysTerms, j = i - k * kBoysTerms;
        tab[i] = a.boys[k * kBoysM + L + j] * kInvFact[j];
    }
    for (int i = threadIdx.x; i < kBoysNT; i += blockDim.x) etab[i] = a.bexp[i];
    __syncthreads();
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= a.ngroups) return;
    const GroupRec g = a.groups[a.g0 + gi];
    double bs[NA][NB], bt[NA][NB], bv[NA][NB];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) bs[i][j] = bt[i][j] = bv[i][j] = 0.0;
    const double w = sqrt(a.w2);
    for (int k = g.pstart; k < g.pend; ++k) {
        const PairRec P = a.pairs[k];
        const double ip = P.pad[0], p = P.p, b = P.pad[1];
        const double h = 0.5 * ip;
        // E with the second index raised by two (kinetic)
        EAxis<LA, LB + 2> Ex, Ey, Ez;
        herm_axis<LA, LB + 2>(h, P.PA[0], P.PB[0], Ex);
        herm_axis<LA, LB + 2>(h, P.PA[1], P.PB[1], Ey);
        herm_axis<LA, LB + 2>(h, P.PA[2], P.PB[2], Ez);
        const double ov = P.cpre * (kPi * ip) * sqrt(kPi * ip);
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int ix = cx(LA, i), iy = cy(LA, i), iz = cz(LA, i);
                const int jx = cx(LB, j), jy = cy(LB, j), jz = cz(LB, j);
                const double ex = Ex.v[ix][jx][0], ey = Ey.v[iy][jy][0], ez = Ez.v[iz][jz][0];
                auto lap = [&](const EAxis<LA, LB + 2> &E, int ii, int jj) {
                    double d = (2 * jj + 1) * b * E.v[ii][jj][0] - 2.0 * b * b * E.v[ii][jj + 2][0];
                    if (jj >= 2) d -= 0.5 * jj * (jj - 1) * E.v[ii][jj - 2][0];
                    return d;
                };
                bs[i][j] += ov * ex * ey * ez;
                bt[i][j] += ov * (lap(Ex, ix, jx) * ey * ez + ex * lap(Ey, iy, jy) * ez + ex * ey * lap(Ez, iz, jz));
            }
        // short-range point-charge sums
        const double c = w * fast_rsqrt(p + a.w2);
        const double arg = P.Cb * 2.0 * kPi * ip * (1.0 - c) * fast_rcp(a.d_ewald_R);
        if (!(arg > 1.0)) continue;
        const double rad2 = (ip + fast_rcp(a.w2)) * screen_log(arg);
        double vs[L + 1][L + 1][L + 1];
#pragma unroll
        for (int t = 0; t <= L; ++t)
#pragma unroll
            for (int u = 0; u <= L - t; ++u)
#pragma unroll
                for (int v = 0; v <= L - t - u; ++v) vs[t][u][v] = 0.0;
        bool any = false;
        for (int C = 0; C < a.natom; ++C) {
            const double qc = a.q[C];
            if (qc == 0.0) continue;
            const double cen[3] = {P.P[0] - a.xyz[3 * C], P.P[1] - a.xyz[3 * C + 1], P.P[2] - a.xyz[3 * C + 2]};
            for_images(a.lat, cen, rad2, a.rcap2, [&](const double *Lv, double L2) {
                double R0[L + 1];
                sr_R0<L, kBoysTerms, true>(p, a.w2, L2, tab, etab, R0);
                double R[L + 1][L + 1][L + 1];
                herm_R<L, double>(R0, Lv[0], Lv[1], Lv[2], R);
#pragma unroll
                for (int t = 0; t <= L; ++t)
#pragma unroll
                    for (int u = 0; u <= L - t; ++u)
#pragma unroll
                        for (int v = 0; v <= L - t - u; ++v) vs[t][u][v] += qc * R[t][u][v];
                any = true;
            });
        }
        if (!any) continue;
        const double pv = P.cpre * 2.0 * kPi * ip;
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int ix = cx(LA, i), iy = cy(LA, i), iz = cz(LA, i);
                const int jx = cx(LB, j), jy = cy(LB, j), jz = cz(LB, j);
                double s = 0.0;
#pragma unroll
                for (int t = 0; t <= ix + jx; ++t)
#pragma unroll
                    for (int u = 0; u <= iy + jy; ++u)
#pragma unroll
                        for (int v = 0; v <= iz + jz; ++v) s += Ex.v[ix][jx][t] * Ey.v[iy][jy][u] * Ez.v[iz][jz][v] * vs[t][u][v];
                bv[i][j] += pv * s;
            }
    }
    const int n = a.nbfc;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const long e = (long)(g.aoA + i) * n + g.aoB + j;
            atomicAdd(&a.XS[e], bs[i][j]);
            atomicAdd(&a.XT[e], bt[i][j]);
            atomicAdd(&a.XV[e], bv[i][j]);
        }
}

// rho[g] = s_g sum_C q_C cos(G.C), rho[ng + g] = -s_g sum_C q_C sin(G.C):
// the nuclear structure factor on the half-space vectors, scaled like the
// pair structure factors (s_g = sqrt of the doubled weight).
__global__ __launch_bounds__(256) void k_rho_nuc(const double *G, const double *Gs, int ng, const double *xyz,
                                                const double *q, int natom, double *rho)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const double gx = G[3 * g], gy = G[3 * g + 1], gz = G[3 * g + 2];
    double re = 0.0, im = 0.0;
    for (int C = 0; C < natom; ++C) {
        double s, c;
        sincos(gx * xyz[3 * C] + gy * xyz[3 * C + 1] + gz * xyz[3 * C + 2], &s, &c);
        re += q[C] * c;
        im -= q[C] * s;
    }
    rho[g] = Gs[g] * re;
    rho[ng + g] = Gs[g] * im;
}

// Real-space part of the point-charge Ewald energy: one thread per ordered
// atom pair (A, B), 1/2 q_A q_B sum_R erfc(w |A - B - R|)/|A - B - R| over
// |A - B - R| < r_bound, R = 0 left out for A = B.
__global__ __launch_bounds__(256) void k_enuc_real(const double *xyz, const double *q, int natom, LatArgs lat,
                                                  double w, double rb2, double *out)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (t < (long)natom * natom) {
        const int A = (int)(t / natom), B = (int)(t % natom);
        const double qq = q[A] * q[B];
        if (qq != 0.0) {
            const double cen[3] = {xyz[3 * A] - xyz[3 * B], xyz[3 * A + 1] - xyz[3 * B + 1],
                                   xyz[3 * A + 2] - xyz[3 * B + 2]};
            for_images(lat, cen, rb2, 0.0, [&](const double *, double L2) {
                if (L2 > 0.0) {
                    const double r = sqrt(L2);
                    e += erfc(w * r) / r;
                }
            });
            e *= 0.5 * qq;
        }
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
    if ((threadIdx.x & 63) == 0 && e != 0.0) atomicAdd(out, e);
}

template <int LA, int LB>
hipError_t launch_one_e_t(const OneEArgs &a, hipStream_t st)
{
    if (a.ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_one_e<LA, LB>), dim3((a.ngroups + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_one_e(int cls, const OneEArgs &a, hipStream_t st)
{
    switch (cls) {
        case 0: return launch_one_e_t<0, 0>(a, st);
        case 1: return launch_one_e_t<1, 0>(a, st);
        case 2: return launch_one_e_t<1, 1>(a, st);
        case 3: return launch_one_e_t<2, 0>(a, st);
        case 4: return launch_one_e_t<2, 1>(a, st);
        default: return launch_one_e_t<2, 2>(a, st);
    }
}

hipError_t launch_rho_nuc(const double *G, const double *Gs, int ng, const double *xyz, const double *q, int natom,
                          double *rho, hipStream_t st)
{
    if (ng <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rho_nuc, dim3((ng + 255) / 256), dim3(256), 0, st, G, Gs, ng, xyz, q, natom, rho);
    return hipGetLastError();
}

hipError_t launch_enuc_real(const double *xyz, const double *q, int natom, const LatArgs &lat, double w,
                            double rb2, double *out, hipStream_t st)
{
    const long n = (long)natom * natom;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_enuc_real, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xyz, q, natom, lat, w, rb2,
                       out);
    return hipGetLastError();
}

}  // namespace pbcjk
