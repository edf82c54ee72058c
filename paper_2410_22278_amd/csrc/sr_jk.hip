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
// Mapping: one lane per entry of the class pair's neighbour list (group
// pairs that have at least one real-space term; entries of one bra group
// are consecutive, so a wavefront mostly shares its bra data).  Each lane
// applies the density-weighted screen, the real-space sphere and the image
// search of every primitive quartet of its group pair.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "kernels.h"

namespace pbcjk {

namespace {

// acc += pref * sum_t E^ab_t sum_s (-1)^|s| E^cd_s R_{t+s}  (ket transform
// first, then the bra), evaluated in the value type V.
template <int LA, int LB, int LC, int LD, typename V>
__device__ __forceinline__ void add_term(const EAxis<LA, LB> &Ex, const EAxis<LA, LB> &Ey, const EAxis<LA, LB> &Ez,
                                         const EAxis<LC, LD> &Fx, const EAxis<LC, LD> &Fy, const EAxis<LC, LD> &Fz,
                                         const V (&R)[LA + LB + LC + LD + 1][LA + LB + LC + LD + 1][LA + LB + LC + LD + 1],
                                         double pref, double (&acc)[ncart(LA)][ncart(LB)][ncart(LC)][ncart(LD)])
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int LAB = LA + LB;
#pragma unroll
    for (int ic = 0; ic < NC; ++ic)
#pragma unroll
        for (int id = 0; id < ND; ++id) {
            const int sx = cx(LC, ic) + cx(LD, id), sy = cy(LC, ic) + cy(LD, id), sz = cz(LC, ic) + cz(LD, id);
            V W[LAB + 1][LAB + 1][LAB + 1];
#pragma unroll
            for (int t = 0; t <= LAB; ++t)
#pragma unroll
                for (int u = 0; u <= LAB - t; ++u)
#pragma unroll
                    for (int v = 0; v <= LAB - t - u; ++v) {
                        V w = V(0);
#pragma unroll
                        for (int tt = 0; tt <= sx; ++tt)
#pragma unroll
                            for (int uu = 0; uu <= sy; ++uu)
#pragma unroll
                                for (int vv = 0; vv <= sz; ++vv) {
                                    const V e = V(Fx.v[cx(LC, ic)][cx(LD, id)][tt] * Fy.v[cy(LC, ic)][cy(LD, id)][uu] *
                                                  Fz.v[cz(LC, ic)][cz(LD, id)][vv]);
                                    const V rv = R[t + tt][u + uu][v + vv];
                                    w += ((tt + uu + vv) & 1) ? -e * rv : e * rv;
                                }
                        W[t][u][v] = w;
                    }
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int ib = 0; ib < NB; ++ib) {
                    const int ax = cx(LA, ia) + cx(LB, ib), ay = cy(LA, ia) + cy(LB, ib), az = cz(LA, ia) + cz(LB, ib);
                    V sacc = V(0);
#pragma unroll
                    for (int t = 0; t <= ax; ++t)
#pragma unroll
                        for (int u = 0; u <= ay; ++u)
#pragma unroll
                            for (int v = 0; v <= az; ++v)
                                sacc += V(Ex.v[cx(LA, ia)][cx(LB, ib)][t] * Ey.v[cy(LA, ia)][cy(LB, ib)][u] *
                                          Ez.v[cz(LA, ia)][cz(LB, ib)][v]) * W[t][u][v];
                    acc[ia][ib][ic][id] += pref * (double)sacc;
                }
        }
}

template <int LA, int LB, int LC, int LD, bool MIX>
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
    const int lane = threadIdx.x & 63;
    const int n = a.nbfc, ns = a.nshell;
    unsigned long long cnt_q = 0, cnt_t = 0, cnt_f = 0;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;

    if (e < a.n_entries) {
        const int bi = a.nbr_bra[e], j = a.nbr_ket[e];
        const GroupRec gb = a.groups[a.gb0 + bi];
        const GroupRec gk = a.groups[a.gk0 + j];
        const int A = gb.shA, B = gb.shB, C = gk.shA, D = gk.shB;
        double wD = a.Dmax[A * ns + B];
        wD = fmax(wD, a.Dmax[C * ns + D]);
        wD = fmax(wD, a.Dmax[A * ns + C]);
        wD = fmax(wD, a.Dmax[A * ns + D]);
        wD = fmax(wD, a.Dmax[B * ns + C]);
        wD = fmax(wD, a.Dmax[B * ns + D]);
        if (gb.Qmax * gk.Qmax * wD > a.d_schwarz) {
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
                double rad2;
                if (!quartet_sphere(Pb, Pk, a.w2, a.d_ewald_R, rad2)) continue;
                const double p = Pb.p, q = Pk.p, pq = p * q;
                const double rho = pq / (p + q);
                const double pref = Pb.cpre * Pk.cpre * kTwoPi52 / (pq * sqrt(p + q));
                EAxis<LC, LD> Fx, Fy, Fz;
                const double hk = 0.5 / q;
                herm_axis<LC, LD>(hk, Pk.PA[0], Pk.PB[0], Fx);
                herm_axis<LC, LD>(hk, Pk.PA[1], Pk.PB[1], Fy);
                herm_axis<LC, LD>(hk, Pk.PA[2], Pk.PB[2], Fz);
                const double cen[3] = {Pb.P[0] - Pk.P[0], Pb.P[1] - Pk.P[1], Pb.P[2] - Pk.P[2]};
                const bool lowp = MIX && (Pb.Q * Pk.Q * wD < a.fp32_below);
                for_images(a.lat, cen, rad2, a.rcap2, [&](const double *Lv, double L2) {
                    ++cnt_t;
                    if (MIX && lowp) {
                        ++cnt_f;
                        float R0[L + 1];
                        sr_R0_mixed<L>(rho, a.w2, L2, tab, R0);
                        float R[L + 1][L + 1][L + 1];
                        herm_R<L, float>(R0, (float)Lv[0], (float)Lv[1], (float)Lv[2], R);
                        add_term<LA, LB, LC, LD, float>(Ex, Ey, Ez, Fx, Fy, Fz, R, pref, acc);
                    } else {
                        double R0[L + 1];
                        sr_R0<L>(rho, a.w2, L2, tab, R0);
                        double R[L + 1][L + 1][L + 1];
                        herm_R<L, double>(R0, Lv[0], Lv[1], Lv[2], R);
                        add_term<LA, LB, LC, LD, double>(Ex, Ey, Ez, Fx, Fy, Fz, R, pref, acc);
                    }
                });
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
    }
    // per-lane counters, summed across the wave before one atomic each
    for (int off = 32; off > 0; off >>= 1) {
        cnt_q += __shfl_down(cnt_q, off, 64);
        cnt_t += __shfl_down(cnt_t, off, 64);
        cnt_f += __shfl_down(cnt_f, off, 64);
    }
    if (lane == 0) {
        atomicAdd(&a.counters[0], cnt_q);
        atomicAdd(&a.counters[1], cnt_t);
        atomicAdd(&a.counters[2 + a.slot], cnt_t);
        if (MIX) atomicAdd(&a.counters[23], cnt_f);
    }
}

template <int LA, int LB, int LC, int LD>
hipError_t launch_one(const SRArgs &a, hipStream_t st)
{
    if (a.n_entries <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.n_entries + 255) / 256)), block(256);
    if (a.fp32_below > 0)
        hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD, false>), grid, block, 0, st, a);
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
    // d-shell class pairs up to total angular momentum 3; larger ones run in
    // the cooperative kernel
    PBCJK_CASE(0, 3) PBCJK_CASE(0, 4) PBCJK_CASE(1, 3)
#endif
#undef PBCJK_CASE
    return hipErrorNotSupported;
}

}  // namespace pbcjk
