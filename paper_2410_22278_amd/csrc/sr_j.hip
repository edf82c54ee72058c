// Short-range Coulomb matrix alone (J-engine), for builds that do not ask
// for K.
//
// The density is first expanded per local primitive pair in the Hermite
// basis of that pair (Sec. 3.2, eqs. pbc_j_split_1 to pbc_j_split_4):
//   D~_t(pair) = cpre sum_{a in A, b in B} E^{ab}_t D[a][b],     t = (t,u,v), |t| <= la + lb,
// (k_hdens; cpre carries the contraction coefficients, normalisations,
// Gaussian factor and symmetry weight of the pair).  A quartet's real-space
// term then contributes to both halves of J without ever forming the
// Cartesian block:
//   X[a,b] += 2w K0 cpre_bra sum_t E^{ab}_t sum_s (-1)^{|s|} R_{t+s} D~_s(ket),
//   X[c,d] += 2w K0 cpre_ket sum_s (-1)^{|s|} E^{cd}_s sum_t R_{t+s} D~_t(bra),
// K0 = 2 pi^{5/2}/(pq sqrt(p+q)), with the same pairs, screens, spheres and
// lattice shifts as the J/K kernel, so J = X + X^T + J_LR + J_self is the
// same sum.  Per quartet that is two n_h(ab) x n_h(cd) contractions instead
// of the Cartesian block and its six scatters.  The ket-side Hermite sums
// are accumulated over the bra primitives of one ket primitive and
// transformed once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sr_lane.h"

namespace pbcjk {

namespace {

__host__ __device__ constexpr int nherm_j(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }

// Hermite index of (t,u,v) within the n_h(L) block: degree-major, then t
// descending, then u descending (the order of k_hdens' output).
__host__ __device__ constexpr int hidx_j(int t, int u, int v)
{
    return (t + u + v) * (t + u + v + 1) * (t + u + v + 2) / 6 + (u + v) * (u + v + 1) / 2 + v;
}

template <int LA, int LB>
__global__ __launch_bounds__(256) void k_hdens(HdensArgs a)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), LAB = LA + LB, NH = nherm_j(LAB);
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= a.ngroups) return;
    const GroupRec g = a.groups[a.g0 + gi];
    const int n = a.nbfc;
    double Dab[NA][NB];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) Dab[i][j] = a.Dt[(long)(g.aoA + i) * n + g.aoB + j];
    for (int k = g.pstart; k < g.pend; ++k) {
        const PairRec P = a.pairs[k];
        EAxis<LA, LB> Ex, Ey, Ez;
        const double h = 0.5 * P.pad[0];
        herm_axis<LA, LB>(h, P.PA[0], P.PB[0], Ex);
        herm_axis<LA, LB>(h, P.PA[1], P.PB[1], Ey);
        herm_axis<LA, LB>(h, P.PA[2], P.PB[2], Ez);
        double out[NH];
#pragma unroll
        for (int q = 0; q < NH; ++q) out[q] = 0.0;
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int ax = cx(LA, i) + cx(LB, j), ay = cy(LA, i) + cy(LB, j), az = cz(LA, i) + cz(LB, j);
#pragma unroll
                for (int t = 0; t <= ax; ++t)
#pragma unroll
                    for (int u = 0; u <= ay; ++u)
#pragma unroll
                        for (int v = 0; v <= az; ++v)
                            out[hidx_j(t, u, v)] += Ex.v[cx(LA, i)][cx(LB, j)][t] * Ey.v[cy(LA, i)][cy(LB, j)][u] *
                                                    Ez.v[cz(LA, i)][cz(LB, j)][v] * Dab[i][j];
            }
        double *o = a.hd + (long)(k - a.p0) * NH;
#pragma unroll
        for (int q = 0; q < NH; ++q) o[q] = P.cpre * out[q];
    }
}

typedef const __attribute__((address_space(4))) double *CDblPtr;

template <int N, class P>
__device__ __forceinline__ void load_vec(P p, double (&v)[N])
{
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = p[q];
}

template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sr_waves_per_eu<LA, LB, LC, LD>())))
void k_sr_j(SRArgs a)
{
    constexpr int L = LA + LB + LC + LD;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int LAB = LA + LB, LCD = LC + LD;
    constexpr int NHB = nherm_j(LAB), NHK = nherm_j(LCD);
    __shared__ double tab[kBoysNT * kBoysTerms];
    __shared__ double etab[kBoysNT];
    // blocks past the work list's device-side length leave before staging
    // the Boys table
    if ((long)blockIdx.x * blockDim.x >= (long)*a.count) return;
    constexpr double kInvFact[kBoysTerms] = {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720,
                                             1.0 / 5040, 1.0 / 40320};
    for (int i = threadIdx.x; i < kBoysNT * kBoysTerms; i += blockDim.x) {
        int k = i / kBoysTerms, jj = i - k * kBoysTerms;
        tab[i] = a.boys[k * kBoysM + L + jj] * kInvFact[jj];
    }
    for (int i = threadIdx.x; i < kBoysNT; i += blockDim.x) etab[i] = a.bexp[i];
    __syncthreads();
    const int ns = a.nshell;
    unsigned long long cnt_q = 0, cnt_t = 0;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;

    if (e < (long)*a.count) {
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
        double acc_ab[NA][NB], acc_cd[NC][ND];
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) acc_ab[i][jj] = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int jj = 0; jj < ND; ++jj) acc_cd[i][jj] = 0.0;
        unsigned long long ent_terms = 0;
        // the nearest lattice translate of the group centres' difference
        // starts each quartet's image search
        double S[3];
        {
            const double cg[3] = {gb.C[0] - gk.C[0], gb.C[1] - gk.C[1], gb.C[2] - gk.C[2]};
            double n[3];
            nearest_translate(a.lat, cg, n);
#pragma unroll
            for (int x = 0; x < 3; ++x) S[x] = n[0] * a.lat.M[x] + n[1] * a.lat.M[3 + x] + n[2] * a.lat.M[6 + x];
        }
        // ket pairs outer, bra pairs inner, as in the J/K kernel (wave-uniform
        // bra records and Hermite densities read through the scalar unit)
        auto run = [&](auto bpairs, auto bhd, int pbs, int pbe) {
            const int pk_end = (gb.Qmax * gk.Qmax * wD > a.d_schwarz) ? gk.pend : gk.pstart;
            for (int pk = gk.pstart; pk < pk_end; ++pk) {
                const PairRec Pk = a.pairs[pk];
                if (!(gb.Qmax * Pk.Q * wD > a.d_schwarz)) break;
                double Dk[NHK];
                load_vec<NHK>(a.hd_k + (long)(pk - a.hd_p0k) * NHK, Dk);
                double Jk[NHK];
#pragma unroll
                for (int q = 0; q < NHK; ++q) Jk[q] = 0.0;
                bool any = false;
                for (int pb = pbs; pb < pbe; ++pb) {
                    const PairRec Pb = load_pair(bpairs + pb);
                    if (!(Pb.Q * Pk.Q * wD > a.d_schwarz)) break;
                    ++cnt_q;
                    double rad2;
                    if (!quartet_sphere(Pb, Pk, a.w2, a.d_ewald_R, rad2)) continue;
                    const double rho = fast_rcp(Pb.pad[0] + Pk.pad[0]);
                    const double cen[3] = {Pb.P[0] - Pk.P[0], Pb.P[1] - Pk.P[1], Pb.P[2] - Pk.P[2]};
                    // lattice sum of the Hermite integrals in FP64 (the contraction is linear in R)
                    double Rs[L + 1][L + 1][L + 1];
#pragma unroll
                    for (int t = 0; t <= L; ++t)
#pragma unroll
                        for (int u = 0; u <= L - t; ++u)
#pragma unroll
                            for (int v = 0; v <= L - t - u; ++v) Rs[t][u][v] = 0.0;
                    int nimg = 0;
                    for_images_from(a.lat, cen, S, rad2, a.rcap2, [&](const double *Lv, double L2) {
                        ++nimg;
                        double R0[L + 1];
                        sr_R0<L, kBoysTerms, true>(rho, a.w2, L2, tab, etab, R0);
                        double R[L + 1][L + 1][L + 1];
                        herm_R<L, double>(R0, Lv[0], Lv[1], Lv[2], R);
#pragma unroll
                        for (int t = 0; t <= L; ++t)
#pragma unroll
                            for (int u = 0; u <= L - t; ++u)
#pragma unroll
                                for (int v = 0; v <= L - t - u; ++v) Rs[t][u][v] += R[t][u][v];
                    });
                    if (nimg == 0) continue;
                    cnt_t += nimg;
                    ent_terms += nimg;
                    any = true;
                    const double K0 = kTwoPi52 * Pb.pad[0] * Pk.pad[0] * fast_rsqrt(Pb.p + Pk.p);
                    double Db[NHB];
                    load_vec<NHB>(bhd + (long)(pb - a.hd_p0b) * NHB, Db);
                    // ket side: Jk_s += K0 cpre_ket (-1)^{|s|} sum_t R_{t+s} D~_t(bra)
                    const double fk = K0 * Pk.cpre;
#pragma unroll
                    for (int tt = 0; tt <= LCD; ++tt)
#pragma unroll
                        for (int uu = 0; uu <= LCD - tt; ++uu)
#pragma unroll
                            for (int vv = 0; vv <= LCD - tt - uu; ++vv) {
                                double sum = 0.0;
#pragma unroll
                                for (int t = 0; t <= LAB; ++t)
#pragma unroll
                                    for (int u = 0; u <= LAB - t; ++u)
#pragma unroll
                                        for (int v = 0; v <= LAB - t - u; ++v)
                                            sum = fma(Rs[t + tt][u + uu][v + vv], Db[hidx_j(t, u, v)], sum);
                                Jk[hidx_j(tt, uu, vv)] += ((tt + uu + vv) & 1) ? -fk * sum : fk * sum;
                            }
                    // bra side: X[a,b] += K0 cpre_bra sum_t E^ab_t sum_s (-1)^{|s|} R_{t+s} D~_s(ket)
                    EAxis<LA, LB> Ex, Ey, Ez;
                    const double hb = 0.5 * Pb.pad[0];
                    herm_axis<LA, LB>(hb, Pb.PA[0], Pb.PB[0], Ex);
                    herm_axis<LA, LB>(hb, Pb.PA[1], Pb.PB[1], Ey);
                    herm_axis<LA, LB>(hb, Pb.PA[2], Pb.PB[2], Ez);
                    double vb[NHB];
#pragma unroll
                    for (int t = 0; t <= LAB; ++t)
#pragma unroll
                        for (int u = 0; u <= LAB - t; ++u)
#pragma unroll
                            for (int v = 0; v <= LAB - t - u; ++v) {
                                double sum = 0.0;
#pragma unroll
                                for (int tt = 0; tt <= LCD; ++tt)
#pragma unroll
                                    for (int uu = 0; uu <= LCD - tt; ++uu)
#pragma unroll
                                        for (int vv = 0; vv <= LCD - tt - uu; ++vv) {
                                            const double r = Rs[t + tt][u + uu][v + vv] * Dk[hidx_j(tt, uu, vv)];
                                            sum += ((tt + uu + vv) & 1) ? -r : r;
                                        }
                                vb[hidx_j(t, u, v)] = sum;
                            }
                    const double fb = K0 * Pb.cpre;
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
                                        s += Ex.v[cx(LA, ia)][cx(LB, ib)][t] * Ey.v[cy(LA, ia)][cy(LB, ib)][u] *
                                             Ez.v[cz(LA, ia)][cz(LB, ib)][v] * vb[hidx_j(t, u, v)];
                            acc_ab[ia][ib] += fb * s;
                        }
                }
                if (any) {
                    // ket transform of this ket primitive's Hermite sums
                    EAxis<LC, LD> Fx, Fy, Fz;
                    const double hk = 0.5 * Pk.pad[0];
                    herm_axis<LC, LD>(hk, Pk.PA[0], Pk.PB[0], Fx);
                    herm_axis<LC, LD>(hk, Pk.PA[1], Pk.PB[1], Fy);
                    herm_axis<LC, LD>(hk, Pk.PA[2], Pk.PB[2], Fz);
#pragma unroll
                    for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                        for (int id = 0; id < ND; ++id) {
                            const int sx = cx(LC, ic) + cx(LD, id), sy = cy(LC, ic) + cy(LD, id),
                                      sz = cz(LC, ic) + cz(LD, id);
                            double s = 0.0;
#pragma unroll
                            for (int tt = 0; tt <= sx; ++tt)
#pragma unroll
                                for (int uu = 0; uu <= sy; ++uu)
#pragma unroll
                                    for (int vv = 0; vv <= sz; ++vv)
                                        s += Fx.v[cx(LC, ic)][cx(LD, id)][tt] * Fy.v[cy(LC, ic)][cy(LD, id)][uu] *
                                             Fz.v[cz(LC, ic)][cz(LD, id)][vv] * Jk[hidx_j(tt, uu, vv)];
                            acc_cd[ic][id] += s;
                        }
                }
            }
        };
        const int bi0 = __builtin_amdgcn_readfirstlane(bi);
        if (__builtin_amdgcn_ballot_w64(bi != bi0) == 0) {
            run((CPairPtr)a.pairs, (CDblPtr)a.hd_b, __builtin_amdgcn_readfirstlane(gb.pstart),
                __builtin_amdgcn_readfirstlane(gb.pend));
        } else {
            run(a.pairs, a.hd_b, gb.pstart, gb.pend);
        }
        if (ent_terms > 0) {
            const double w2 = 2.0 * ((a.tri && j == bi) ? 0.5 : 1.0);
            const int n = a.nbfc;
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int ib = 0; ib < NB; ++ib) atomicAdd(&a.X[(gb.aoA + ia) * n + gb.aoB + ib], w2 * acc_ab[ia][ib]);
#pragma unroll
            for (int ic = 0; ic < NC; ++ic)
#pragma unroll
                for (int id = 0; id < ND; ++id) atomicAdd(&a.X[(gk.aoA + ic) * n + gk.aoB + id], w2 * acc_cd[ic][id]);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        cnt_q += __shfl_down(cnt_q, off, 64);
        cnt_t += __shfl_down(cnt_t, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&a.counters[0], cnt_q);
        atomicAdd(&a.counters[1], cnt_t);
        atomicAdd(&a.counters[2 + a.slot], cnt_t);
        atomicAdd(&a.counters[24 + a.slot], cnt_q);
    }
}

constexpr int kLaJ[kNumClass] = {0, 1, 1, 2, 2, 2};
constexpr int kLbJ[kNumClass] = {0, 0, 1, 0, 1, 2};

template <int LA, int LB>
hipError_t launch_hdens_t(const HdensArgs &a, hipStream_t st)
{
    if (a.ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_hdens<LA, LB>), dim3((a.ngroups + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int CB, int CK>
hipError_t launch_j_pair(const SRArgs &a, hipStream_t st)
{
    if (a.max_entries <= 0) return hipSuccess;
    const dim3 g((unsigned)std::max(1L, (a.max_entries + 255) / 256)), b(256);
    hipLaunchKernelGGL((k_sr_j<kLaJ[CB], kLbJ[CB], kLaJ[CK], kLbJ[CK]>), g, b, 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hdens(int cls, const HdensArgs &a, hipStream_t st)
{
    switch (cls) {
        case 0: return launch_hdens_t<0, 0>(a, st);
        case 1: return launch_hdens_t<1, 0>(a, st);
        case 2: return launch_hdens_t<1, 1>(a, st);
        case 3: return launch_hdens_t<2, 0>(a, st);
        case 4: return launch_hdens_t<2, 1>(a, st);
        default: return launch_hdens_t<2, 2>(a, st);
    }
}

// Class pairs (cb <= ck) with total angular momentum up to 6; others return
// hipErrorNotSupported (the caller runs the J/K kernel for them).
hipError_t launch_sr_j(int cb, int ck, const SRArgs &a, hipStream_t st)
{
#define PBCJK_JCASE(X, Y) \
    if (cb == X && ck == Y) return launch_j_pair<X, Y>(a, st);
    PBCJK_JCASE(0, 0) PBCJK_JCASE(0, 1) PBCJK_JCASE(0, 2) PBCJK_JCASE(1, 1) PBCJK_JCASE(1, 2) PBCJK_JCASE(2, 2)
#if PBCJK_WITH_D
    PBCJK_JCASE(0, 3) PBCJK_JCASE(0, 4) PBCJK_JCASE(0, 5) PBCJK_JCASE(1, 3) PBCJK_JCASE(1, 4) PBCJK_JCASE(1, 5)
    PBCJK_JCASE(2, 3) PBCJK_JCASE(2, 4) PBCJK_JCASE(3, 3) PBCJK_JCASE(3, 4)
#endif
#undef PBCJK_JCASE
    return hipErrorNotSupported;
}

}  // namespace pbcjk
