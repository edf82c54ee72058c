// Short-range (real-space erfc) part of the Gamma-point J and K builds.
//
// For each unique pair of (shell pair, image) groups the kernel sums the
// primitive quartets and the lattice shifts R1 of the ket (Sec. 2.4, eq.
// pbc_eri_general_final, real-space term) into a contracted Cartesian
// integral block held in registers, then contracts the block with the
// density into the J and K halves:
//   X[a,b] += 2w I D[c,d],  X[c,d] += 2w I D[a,b]          (J = X + X^T)
//   Y[a,c] += w I D[b,d], Y[b,c] += w I D[a,d],
//   Y[a,d] += w I D[b,c], Y[b,d] += w I D[a,c]              (K = Y + Y^T)
// with w = 1/2 on the diagonal group pair and 1 otherwise (the primitive
// symmetry weights are folded into the pair prefactors).
//
// Mapping: one wavefront per bra group, 64 lanes over the ket groups of one
// class whose Cauchy-Schwarz value can pass the density-weighted screen
// (the ket list is sorted by that value, so the candidates form a prefix).
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "kernels.h"

namespace pbcjk {

namespace {

constexpr double kTwoPi52 = 34.98683665524972497;   // 2 pi^{5/2}

template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(256) void k_sr_jk(SRArgs a)
{
    constexpr int L = LA + LB + LC + LD;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int LAB = LA + LB;
    __shared__ double tab[kBoysNT * kBoysTerms];
    for (int i = threadIdx.x; i < kBoysNT * kBoysTerms; i += blockDim.x) {
        int k = i / kBoysTerms, j = i - k * kBoysTerms;
        tab[i] = a.boys[k * kBoysM + L + j];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bi = blockIdx.x * (blockDim.x >> 6) + wave;
    if (bi >= a.nb) return;
    const GroupRec gb = a.groups[a.gb0 + bi];
    const double dglob = *a.dmax_glob;
    const double qthr = a.d_schwarz / (gb.Qmax * dglob);
    int lo = 0, hi = a.nk;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a.groups[a.gk0 + mid].Qmax > qthr) lo = mid + 1; else hi = mid;
    }
    const int jhi = lo;
    const int jlo = a.tri ? bi : 0;
    const int n = a.nbfc, ns = a.nshell;
    unsigned long long cnt_q = 0, cnt_t = 0;

    for (int j = jlo + lane; j < jhi; j += 64) {
        const GroupRec gk = a.groups[a.gk0 + j];
        const int A = gb.shA, B = gb.shB, C = gk.shA, D = gk.shB;
        double wD = a.Dmax[A * ns + B];
        wD = fmax(wD, a.Dmax[C * ns + D]);
        wD = fmax(wD, a.Dmax[A * ns + C]);
        wD = fmax(wD, a.Dmax[A * ns + D]);
        wD = fmax(wD, a.Dmax[B * ns + C]);
        wD = fmax(wD, a.Dmax[B * ns + D]);
        if (!(gb.Qmax * gk.Qmax * wD > a.d_schwarz)) continue;

        double acc[NA][NB][NC][ND];
#pragma unroll
        for (int i0 = 0; i0 < NA; ++i0)
#pragma unroll
            for (int i1 = 0; i1 < NB; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < NC; ++i2)
#pragma unroll
                    for (int i3 = 0; i3 < ND; ++i3) acc[i0][i1][i2][i3] = 0.0;

        for (int pb = gb.pstart; pb < gb.pend; ++pb) {
            const PairRec Pb = a.pairs[pb];
            EAxis<LA, LB> Ex, Ey, Ez;
            const double hb = 0.5 / Pb.p;
            herm_axis<LA, LB>(hb, Pb.PA[0], Pb.PB[0], Ex);
            herm_axis<LA, LB>(hb, Pb.PA[1], Pb.PB[1], Ey);
            herm_axis<LA, LB>(hb, Pb.PA[2], Pb.PB[2], Ez);
            for (int pk = gk.pstart; pk < gk.pend; ++pk) {
                const PairRec Pk = a.pairs[pk];
                if (!(Pb.Q * Pk.Q * wD > a.d_schwarz)) continue;
                ++cnt_q;
                const double p = Pb.p, q = Pk.p, pq = p * q;
                const double rho = pq / (p + q);
                const double spq = sqrt(p + q);
                const double c = sqrt(a.w2 / (rho + a.w2));
                // real-space sphere of the quartet (Sec. 2.4, eq.
                // pbc_eri_real_cutoff_implementation)
                const double C2e = Pb.Cb * Pk.Cb * kTwoPi52 / (pq * spq);
                const double arg = C2e * (1.0 - c) / a.d_ewald_R;
                if (!(arg > 1.0)) continue;
                const double rad2 = (1.0 / p + 1.0 / q + 1.0 / a.w2) * log(arg);
                const double pref = Pb.cpre * Pk.cpre * kTwoPi52 / (pq * spq);
                EAxis<LC, LD> Fx, Fy, Fz;
                const double hk = 0.5 / q;
                herm_axis<LC, LD>(hk, Pk.PA[0], Pk.PB[0], Fx);
                herm_axis<LC, LD>(hk, Pk.PA[1], Pk.PB[1], Fy);
                herm_axis<LC, LD>(hk, Pk.PA[2], Pk.PB[2], Fz);
                const double cen[3] = {Pb.P[0] - Pk.P[0], Pb.P[1] - Pk.P[1], Pb.P[2] - Pk.P[2]};
                const double r = sqrt(rad2) * (1.0 + 1e-9) + 1e-9;
                int nlo[3], nhi[3];
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    double f = cen[0] * a.Minv[x] + cen[1] * a.Minv[3 + x] + cen[2] * a.Minv[6 + x];
                    nlo[x] = (int)floor(f - r * a.span[x]);
                    nhi[x] = (int)ceil(f + r * a.span[x]);
                }
                for (int n0 = nlo[0]; n0 <= nhi[0]; ++n0)
                    for (int n1 = nlo[1]; n1 <= nhi[1]; ++n1)
                        for (int n2 = nlo[2]; n2 <= nhi[2]; ++n2) {
                            double Lv[3];
#pragma unroll
                            for (int x = 0; x < 3; ++x)
                                Lv[x] = cen[x] - (n0 * a.M[x] + n1 * a.M[3 + x] + n2 * a.M[6 + x]);
                            const double L2 = Lv[0] * Lv[0] + Lv[1] * Lv[1] + Lv[2] * Lv[2];
                            if (!(L2 < rad2)) continue;
                            if (a.rcap2 > 0 && L2 > a.rcap2) continue;
                            ++cnt_t;
                            double R0[L + 1];
                            sr_R0<L>(rho, a.w2, L2, tab, R0);
                            double R[L + 1][L + 1][L + 1];
                            herm_R<L>(R0, Lv[0], Lv[1], Lv[2], R);
                            // ket transform, then bra: sum_t E^ab_t sum_s (-1)^|s| E^cd_s R_{t+s}
#pragma unroll
                            for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                                for (int id = 0; id < ND; ++id) {
                                    const int sx = cx(LC, ic) + cx(LD, id), sy = cy(LC, ic) + cy(LD, id),
                                              sz = cz(LC, ic) + cz(LD, id);
                                    double W[LAB + 1][LAB + 1][LAB + 1];
#pragma unroll
                                    for (int t = 0; t <= LAB; ++t)
#pragma unroll
                                        for (int u = 0; u <= LAB - t; ++u)
#pragma unroll
                                            for (int v = 0; v <= LAB - t - u; ++v) {
                                                double w = 0.0;
#pragma unroll
                                                for (int tt = 0; tt <= sx; ++tt)
#pragma unroll
                                                    for (int uu = 0; uu <= sy; ++uu)
#pragma unroll
                                                        for (int vv = 0; vv <= sz; ++vv) {
                                                            const double e = Fx.v[cx(LC, ic)][cx(LD, id)][tt] *
                                                                             Fy.v[cy(LC, ic)][cy(LD, id)][uu] *
                                                                             Fz.v[cz(LC, ic)][cz(LD, id)][vv];
                                                            const double rv = R[t + tt][u + uu][v + vv];
                                                            w += ((tt + uu + vv) & 1) ? -e * rv : e * rv;
                                                        }
                                                W[t][u][v] = w;
                                            }
#pragma unroll
                                    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                                        for (int ib = 0; ib < NB; ++ib) {
                                            const int ax = cx(LA, ia) + cx(LB, ib), ay = cy(LA, ia) + cy(LB, ib),
                                                      az = cz(LA, ia) + cz(LB, ib);
                                            double s = 0.0;
#pragma unroll
                                            for (int t = 0; t <= ax; ++t)
#pragma unroll
                                                for (int u = 0; u <= ay; ++u)
#pragma unroll
                                                    for (int v = 0; v <= az; ++v)
                                                        s += Ex.v[cx(LA, ia)][cx(LB, ib)][t] *
                                                             Ey.v[cy(LA, ia)][cy(LB, ib)][u] *
                                                             Ez.v[cz(LA, ia)][cz(LB, ib)][v] * W[t][u][v];
                                            acc[ia][ib][ic][id] += pref * s;
                                        }
                                }
                        }
            }
        }

        // contraction with the density and accumulation of the J, K halves
        const double w = (a.tri && j == bi) ? 0.5 : 1.0;
        const double *Dt = a.Dt;
        const int aoA = gb.aoA, aoB = gb.aoB, aoC = gk.aoA, aoD = gk.aoB;
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) {
                double s = 0.0;
#pragma unroll
                for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                    for (int id = 0; id < ND; ++id) s += acc[ia][ib][ic][id] * Dt[(aoC + ic) * n + aoD + id];
                atomicAdd(&a.X[(aoA + ia) * n + aoB + ib], 2.0 * w * s);
            }
#pragma unroll
        for (int ic = 0; ic < NC; ++ic)
#pragma unroll
            for (int id = 0; id < ND; ++id) {
                double s = 0.0;
#pragma unroll
                for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                    for (int ib = 0; ib < NB; ++ib) s += acc[ia][ib][ic][id] * Dt[(aoA + ia) * n + aoB + ib];
                atomicAdd(&a.X[(aoC + ic) * n + aoD + id], 2.0 * w * s);
            }
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ic = 0; ic < NC; ++ic) {
                double s = 0.0;
#pragma unroll
                for (int ib = 0; ib < NB; ++ib)
#pragma unroll
                    for (int id = 0; id < ND; ++id) s += acc[ia][ib][ic][id] * Dt[(aoB + ib) * n + aoD + id];
                atomicAdd(&a.Y[(aoA + ia) * n + aoC + ic], w * s);
            }
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
            for (int ic = 0; ic < NC; ++ic) {
                double s = 0.0;
#pragma unroll
                for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                    for (int id = 0; id < ND; ++id) s += acc[ia][ib][ic][id] * Dt[(aoA + ia) * n + aoD + id];
                atomicAdd(&a.Y[(aoB + ib) * n + aoC + ic], w * s);
            }
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int id = 0; id < ND; ++id) {
                double s = 0.0;
#pragma unroll
                for (int ib = 0; ib < NB; ++ib)
#pragma unroll
                    for (int ic = 0; ic < NC; ++ic) s += acc[ia][ib][ic][id] * Dt[(aoB + ib) * n + aoC + ic];
                atomicAdd(&a.Y[(aoA + ia) * n + aoD + id], w * s);
            }
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
            for (int id = 0; id < ND; ++id) {
                double s = 0.0;
#pragma unroll
                for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                    for (int ic = 0; ic < NC; ++ic) s += acc[ia][ib][ic][id] * Dt[(aoA + ia) * n + aoC + ic];
                atomicAdd(&a.Y[(aoB + ib) * n + aoD + id], w * s);
            }
    }
    // per-lane counters, summed across the wave before one atomic each
    for (int off = 32; off > 0; off >>= 1) {
        cnt_q += __shfl_down(cnt_q, off, 64);
        cnt_t += __shfl_down(cnt_t, off, 64);
    }
    if (lane == 0) {
        atomicAdd(&a.counters[0], cnt_q);
        atomicAdd(&a.counters[1], cnt_t);
    }
}

template <int LA, int LB, int LC, int LD>
hipError_t launch_one(const SRArgs &a, hipStream_t st)
{
    if (a.nb <= 0 || a.nk <= 0) return hipSuccess;
    dim3 grid((a.nb + 3) / 4), block(256);
    hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD>), grid, block, 0, st, a);
    return hipGetLastError();
}

constexpr int kLa[kNumClass] = {0, 1, 1, 2, 2, 2};
constexpr int kLb[kNumClass] = {0, 0, 1, 0, 1, 2};

template <int CB, int CK>
hipError_t launch_pair(const SRArgs &a, hipStream_t st)
{
    return launch_one<kLa[CB], kLb[CB], kLa[CK], kLb[CK]>(a, st);
}

}  // namespace

// Launches the kernel of bra class cb and ket class ck (cb <= ck).
hipError_t launch_sr_jk(int cb, int ck, const SRArgs &a, hipStream_t st)
{
#define PBCJK_CASE(X, Y) \
    if (cb == X && ck == Y) return launch_pair<X, Y>(a, st);
    PBCJK_CASE(0, 0) PBCJK_CASE(0, 1) PBCJK_CASE(0, 2) PBCJK_CASE(1, 1) PBCJK_CASE(1, 2) PBCJK_CASE(2, 2)
#if PBCJK_WITH_D
    PBCJK_CASE(0, 3) PBCJK_CASE(0, 4) PBCJK_CASE(0, 5) PBCJK_CASE(1, 3) PBCJK_CASE(1, 4) PBCJK_CASE(1, 5)
    PBCJK_CASE(2, 3) PBCJK_CASE(2, 4) PBCJK_CASE(2, 5) PBCJK_CASE(3, 3) PBCJK_CASE(3, 4) PBCJK_CASE(3, 5)
    PBCJK_CASE(4, 4) PBCJK_CASE(4, 5) PBCJK_CASE(5, 5)
#endif
#undef PBCJK_CASE
    return hipErrorNotSupported;
}

}  // namespace pbcjk
