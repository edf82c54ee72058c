// Per-lane short-range kernel template (one lane per work-list entry), shared
// by the translation units that instantiate it.  See sr_jk.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.h"
#include "kernels.h"

namespace pbcjk {

namespace {

// Pair records seen through the constant address space (read-only for the
// whole kernel), so that loads at wavefront-uniform addresses go through the
// scalar unit.
typedef const __attribute__((address_space(4))) PairRec *CPairPtr;

__device__ __forceinline__ PairRec load_pair(const PairRec *p) { return *p; }
__device__ __forceinline__ PairRec load_pair(CPairPtr p)
{
    PairRec r;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        r.P[x] = p->P[x];
        r.PA[x] = p->PA[x];
        r.PB[x] = p->PB[x];
        r.pad[x] = p->pad[x];
    }
    r.p = p->p; r.cpre = p->cpre; r.Q = p->Q; r.Cb = p->Cb;
    return r;
}

// acc += pref * sum_t E^ab_t sum_s (-1)^|s| E^cd_s R_{t+s}  (ket transform
// first, then the bra), evaluated in the value type V.
template <int LA, int LB, int LC, int LD, typename V, int IC0, int NIC, typename EV>
__device__ __forceinline__ void add_term(const EAxis<LA, LB, EV> &Ex, const EAxis<LA, LB, EV> &Ey,
                                         const EAxis<LA, LB, EV> &Ez, const EAxis<LC, LD, EV> &Fx,
                                         const EAxis<LC, LD, EV> &Fy, const EAxis<LC, LD, EV> &Fz,
                                         const V (&R)[LA + LB + LC + LD + 1][LA + LB + LC + LD + 1][LA + LB + LC + LD + 1],
                                         double pref, double (&acc)[ncart(LA)][ncart(LB)][NIC][ncart(LD)])
{
    constexpr int NA = ncart(LA), NB = ncart(LB), ND = ncart(LD);
    constexpr int LAB = LA + LB;
#pragma unroll
    for (int icl = 0; icl < NIC; ++icl)
#pragma unroll
        for (int id = 0; id < ND; ++id) {
            const int ic = IC0 + icl;
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
                    acc[ia][ib][icl][id] += pref * (double)sacc;
                }
        }
}

// The bra-block part of J: jab[ia][ib] = 2 w sum_cd acc[ia][ib][c][d] D_cd.
template <int LA, int LB, int LC, int LD, int IC0, int NIC>
__device__ __forceinline__ void contract_ab(const SRArgs &a, const double (&acc)[ncart(LA)][ncart(LB)][NIC][ncart(LD)],
                                            double w, int aoC, int aoD, double (&jab)[ncart(LA)][ncart(LB)])
{
    constexpr int NA = ncart(LA), NB = ncart(LB), ND = ncart(LD);
    const double *Dt = a.Dt;
    const int n = a.nbfc;
    aoC += IC0;
#pragma unroll
    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
            double s = 0.0;
#pragma unroll
            for (int ic = 0; ic < NIC; ++ic)
#pragma unroll
                for (int id = 0; id < ND; ++id) s += acc[ia][ib][ic][id] * Dt[(aoC + ic) * n + aoD + id];
            jab[ia][ib] = 2.0 * w * s;
        }
}

// Adds the density contractions of one contracted block (components
// IC0 .. IC0+NIC-1 of the first ket shell) into the J and K halves (hardware
// FP64 atomics), except the bra block of J (contract_ab), which the caller
// adds; blocks of several slices add up to the full contraction.
template <int LA, int LB, int LC, int LD, int IC0, int NIC>
__device__ __forceinline__ void scatter_block(const SRArgs &a, const double (&acc)[ncart(LA)][ncart(LB)][NIC][ncart(LD)],
                                              double w, int aoA, int aoB, int aoC, int aoD)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), ND = ncart(LD);
    const double *Dt = a.Dt;
    const int n = a.nbfc;
    aoC += IC0;
#pragma unroll
    for (int ic = 0; ic < NIC; ++ic)
#pragma unroll
        for (int id = 0; id < ND; ++id) {
            double s = 0.0;
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int ib = 0; ib < NB; ++ib) s += acc[ia][ib][ic][id] * Dt[(aoA + ia) * n + aoB + ib];
            atomicAdd(&a.X[(aoC + ic) * n + aoD + id], 2.0 * w * s);
        }
    if (!a.want_k) return;   // builds without K: the J targets only
#pragma unroll
    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
        for (int ic = 0; ic < NIC; ++ic) {
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
        for (int ic = 0; ic < NIC; ++ic) {
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
                for (int ic = 0; ic < NIC; ++ic) s += acc[ia][ib][ic][id] * Dt[(aoB + ib) * n + aoC + ic];
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
                for (int ic = 0; ic < NIC; ++ic) s += acc[ia][ib][ic][id] * Dt[(aoA + ia) * n + aoC + ic];
            atomicAdd(&a.Y[(aoB + ib) * n + aoD + id], w * s);
        }
}

// One ket primitive pair Pk against the bra pairs [pbs, pbe) of a group,
// which are stored by descending Q, so the first one that fails the
// Cauchy-Schwarz test ends the sweep.  Per quartet: the density-weighted
// screen, the real-space sphere, the lattice shifts inside it (searched from
// the lattice translate S of the entry's group centres), and the block
// accumulation into acc (see k_sr_jk).
template <int LA, int LB, int LC, int LD, typename V, bool FOLD, int IC0, int NIC, class BP>
__device__ __forceinline__ void bra_sweep(const SRArgs &a, BP bpairs, int pbs, int pbe, const PairRec &Pk, double wD,
                                          const double (&S)[3], const double *tab, const double *etab,
                                          double (&acc)[ncart(LA)][ncart(LB)][NIC][ncart(LD)],
                                          unsigned long long &cnt_q, unsigned long long &cnt_t,
                                          unsigned long long &ent_terms)
{
    constexpr int L = LA + LB + LC + LD;
    constexpr bool F32 = sizeof(V) == 4;
    // E coefficients in the list's precision (FP32 ones take half the registers)
    typedef V EV;
    EAxis<LC, LD, EV> Fx, Fy, Fz;
    const EV hk = EV(0.5 * Pk.pad[0]);
    herm_axis<LC, LD, EV>(hk, EV(Pk.PA[0]), EV(Pk.PB[0]), Fx);
    herm_axis<LC, LD, EV>(hk, EV(Pk.PA[1]), EV(Pk.PB[1]), Fy);
    herm_axis<LC, LD, EV>(hk, EV(Pk.PA[2]), EV(Pk.PB[2]), Fz);
    for (int pb = pbs; pb < pbe; ++pb) {
        const PairRec Pb = load_pair(bpairs + pb);
        if (!(Pb.Q * Pk.Q * wD > a.d_schwarz)) break;
        ++cnt_q;
        double rad2;
        if (!quartet_sphere(Pb, Pk, a.w2, a.d_ewald_R, rad2)) continue;
        const double p = Pb.p, q = Pk.p;
        const double rho = fast_rcp(Pb.pad[0] + Pk.pad[0]);
        const double pref = Pb.cpre * Pk.cpre * kTwoPi52 * Pb.pad[0] * Pk.pad[0] * fast_rsqrt(p + q);
        EAxis<LA, LB, EV> Ex, Ey, Ez;
        const EV hb = EV(0.5 * Pb.pad[0]);
        herm_axis<LA, LB, EV>(hb, EV(Pb.PA[0]), EV(Pb.PB[0]), Ex);
        herm_axis<LA, LB, EV>(hb, EV(Pb.PA[1]), EV(Pb.PB[1]), Ey);
        herm_axis<LA, LB, EV>(hb, EV(Pb.PA[2]), EV(Pb.PB[2]), Ez);
        const double cen[3] = {Pb.P[0] - Pk.P[0], Pb.P[1] - Pk.P[1], Pb.P[2] - Pk.P[2]};
        if (FOLD) {
            // lattice sum of the Hermite integrals in FP64, one transform
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
                if (F32) {
                    float R0[L + 1];
                    sr_R0_f32<L>(rho, a.w2, L2, tab, R0);
                    float R[L + 1][L + 1][L + 1];
                    herm_R<L, float>(R0, (float)Lv[0], (float)Lv[1], (float)Lv[2], R);
#pragma unroll
                    for (int t = 0; t <= L; ++t)
#pragma unroll
                        for (int u = 0; u <= L - t; ++u)
#pragma unroll
                            for (int v = 0; v <= L - t - u; ++v) Rs[t][u][v] += (double)R[t][u][v];
                } else {
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
                }
            });
            if (nimg == 0) continue;
            cnt_t += nimg;
            ent_terms += nimg;
            V Rv[L + 1][L + 1][L + 1];
#pragma unroll
            for (int t = 0; t <= L; ++t)
#pragma unroll
                for (int u = 0; u <= L - t; ++u)
#pragma unroll
                    for (int v = 0; v <= L - t - u; ++v) Rv[t][u][v] = (V)Rs[t][u][v];
            add_term<LA, LB, LC, LD, V, IC0, NIC, EV>(Ex, Ey, Ez, Fx, Fy, Fz, Rv, pref, acc);
        } else {
            for_images_from(a.lat, cen, S, rad2, a.rcap2, [&](const double *Lv, double L2) {
                ++cnt_t;
                ++ent_terms;
                if (F32) {
                    float R0[L + 1];
                    sr_R0_f32<L>(rho, a.w2, L2, tab, R0);
                    float R[L + 1][L + 1][L + 1];
                    herm_R<L, float>(R0, (float)Lv[0], (float)Lv[1], (float)Lv[2], R);
                    add_term<LA, LB, LC, LD, float, IC0, NIC, EV>(Ex, Ey, Ez, Fx, Fy, Fz, R, pref, acc);
                } else {
                    double R0[L + 1];
                    sr_R0<L, kBoysTerms, true>(rho, a.w2, L2, tab, etab, R0);
                    double R[L + 1][L + 1][L + 1];
                    herm_R<L, double>(R0, Lv[0], Lv[1], Lv[2], R);
                    add_term<LA, LB, LC, LD, double, IC0, NIC, EV>(Ex, Ey, Ez, Fx, Fy, Fz, R, pref, acc);
                }
            });
        }
    }
}

// Boys table rows L .. L + kBoysTerms - 1 into LDS, pre-divided by j! so
// that the Taylor sum needs one FMA a term.
template <int L>
__device__ __forceinline__ void load_boys_table(const SRArgs &a, double *tab, double *etab)
{
    constexpr double kInvFact[kBoysTerms] = {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720,
                                             1.0 / 5040, 1.0 / 40320};
    for (int i = threadIdx.x; i < kBoysNT * kBoysTerms; i += blockDim.x) {
        int k = i / kBoysTerms, j = i - k * kBoysTerms;
        tab[i] = a.boys[k * kBoysM + L + j] * kInvFact[j];
    }
    for (int i = threadIdx.x; i < kBoysNT; i += blockDim.x) etab[i] = a.bexp[i];
    __syncthreads();
}

// IC0, NIC: the slice of the first ket shell's Cartesian components whose
// block entries this launch accumulates (the whole shell by default; large d
// class pairs run one launch per slice so that the slice fits in registers,
// each recomputing the shifts' Hermite integrals).  Counters are kept by the
// slice that starts at component 0.
// Wavefronts per SIMD asked of the register allocator, by total angular
// momentum: these kernels wait on dependent FP64 chains (Horner steps, Newton
// steps) and on loads, so more resident wavefronts pay even at the price of
// a few spilled registers (L <= 3); from L = 4 on the spills cost more.
template <int LA, int LB, int LC, int LD>
constexpr int sr_waves_per_eu()
{
    constexpr int L = LA + LB + LC + LD;
    return L == 0 ? 5 : L == 1 ? 4 : L == 2 ? 3 : L == 3 ? 2 : 1;
}

template <int LA, int LB, int LC, int LD, typename V, bool FOLD, int IC0 = 0, int NIC = ncart(LC)>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sr_waves_per_eu<LA, LB, LC, LD>())))
void k_sr_jk(SRArgs a)
{
    constexpr int L = LA + LB + LC + LD;
    constexpr int NA = ncart(LA), NB = ncart(LB), ND = ncart(LD);
    constexpr bool COUNT = IC0 == 0;
    constexpr bool F32 = sizeof(V) == 4;
    // blocks past the work list's device-side length (the grid is sized by
    // the host-side upper bound) leave before staging the Boys table
    if ((long)blockIdx.x * blockDim.x >= (long)*a.count) return;
    __shared__ double tab[kBoysNT * kBoysTerms];
    __shared__ double etab[kBoysNT];
    load_boys_table<L>(a, tab, etab);
    const int lane = threadIdx.x & 63;
    const int ns = a.nshell;
    unsigned long long cnt_q = 0, cnt_t = 0;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool have = e < (long)*a.count;
    const int bi = have ? a.nbr_bra[e] : -1;
    // all lanes hold one bra group (the usual case: the lists run in bra order)
    const int bi0 = __builtin_amdgcn_readfirstlane(bi);
    const bool uni = __builtin_amdgcn_ballot_w64(have && bi != bi0) == 0;
    double jab[NA][NB];
#pragma unroll
    for (int i0 = 0; i0 < NA; ++i0)
#pragma unroll
        for (int i1 = 0; i1 < NB; ++i1) jab[i0][i1] = 0.0;
    int aoA = 0, aoB = 0;

    if (have) {
        const int j = a.nbr_ket[e];
        const GroupRec gb = a.groups[a.gb0 + bi];
        const GroupRec gk = a.groups[a.gk0 + j];
        const int A = gb.shA, B = gb.shB, C = gk.shA, D = gk.shB;
        aoA = gb.aoA;
        aoB = gb.aoB;
        double wD = a.Dmax[A * ns + B];
        wD = fmax(wD, a.Dmax[C * ns + D]);
        wD = fmax(wD, a.Dmax[A * ns + C]);
        wD = fmax(wD, a.Dmax[A * ns + D]);
        wD = fmax(wD, a.Dmax[B * ns + C]);
        wD = fmax(wD, a.Dmax[B * ns + D]);
        double acc[NA][NB][NIC][ND];
#pragma unroll
        for (int i0 = 0; i0 < NA; ++i0)
#pragma unroll
            for (int i1 = 0; i1 < NB; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < NIC; ++i2)
#pragma unroll
                    for (int i3 = 0; i3 < ND; ++i3) acc[i0][i1][i2][i3] = 0.0;
        unsigned long long ent_terms = 0;
        // the nearest lattice translate of the group centres' difference
        double S[3];
        {
            const double cg[3] = {gb.C[0] - gk.C[0], gb.C[1] - gk.C[1], gb.C[2] - gk.C[2]};
            double n[3];
            nearest_translate(a.lat, cg, n);
#pragma unroll
            for (int x = 0; x < 3; ++x) S[x] = n[0] * a.lat.M[x] + n[1] * a.lat.M[3 + x] + n[2] * a.lat.M[6 + x];
        }
        // Ket pairs outer (each lane reads its own ket records once), bra pairs
        // inner.  A group's pairs are stored by descending Q, so the first pair
        // that fails the Cauchy-Schwarz test ends its loop.  When every lane of
        // the wavefront has the same bra group, the bra records are read
        // through the constant address space, so their loads are scalar and the
        // bra loop is uniform.
        auto run = [&](auto bpairs, int pbs, int pbe) {
            const int pk_end = (gb.Qmax * gk.Qmax * wD > a.d_schwarz) ? gk.pend : gk.pstart;
            for (int pk = gk.pstart; pk < pk_end; ++pk) {
                const PairRec Pk = a.pairs[pk];
                if (!(gb.Qmax * Pk.Q * wD > a.d_schwarz)) break;
                bra_sweep<LA, LB, LC, LD, V, FOLD, IC0, NIC>(a, bpairs, pbs, pbe, Pk, wD, S, tab, etab, acc, cnt_q,
                                                            cnt_t, ent_terms);
            }
        };
        if (uni) {
            const CPairPtr cp = (CPairPtr)a.pairs;
            run(cp, __builtin_amdgcn_readfirstlane(gb.pstart), __builtin_amdgcn_readfirstlane(gb.pend));
        } else {
            run(a.pairs, gb.pstart, gb.pend);
        }
        if (ent_terms > 0) {
            const double w = (a.tri && j == bi) ? 0.5 : 1.0;
            contract_ab<LA, LB, LC, LD, IC0, NIC>(a, acc, w, gk.aoA, gk.aoB, jab);
            scatter_block<LA, LB, LC, LD, IC0, NIC>(a, acc, w, gb.aoA, gb.aoB, gk.aoA, gk.aoB);
        }
    }
    // The bra block of J: with one bra group in the wavefront, summed across
    // the lanes before one atomic per element; otherwise per lane.
    {
        const int n = a.nbfc;
        if (uni) {
            const int ra = __builtin_amdgcn_readfirstlane(aoA), rb = __builtin_amdgcn_readfirstlane(aoB);
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int ib = 0; ib < NB; ++ib) {
                    double v = jab[ia][ib];
                    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                    if (lane == 0 && v != 0.0) atomicAdd(&a.X[(ra + ia) * n + rb + ib], v);
                }
        } else if (have) {
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int ib = 0; ib < NB; ++ib)
                    if (jab[ia][ib] != 0.0) atomicAdd(&a.X[(aoA + ia) * n + aoB + ib], jab[ia][ib]);
        }
    }
    // per-lane counters, summed across the wave before one atomic each
    for (int off = 32; off > 0; off >>= 1) {
        cnt_q += __shfl_down(cnt_q, off, 64);
        cnt_t += __shfl_down(cnt_t, off, 64);
    }
    if (COUNT && lane == 0) {
        atomicAdd(&a.counters[0], cnt_q);
        atomicAdd(&a.counters[1], cnt_t);
        atomicAdd(&a.counters[2 + a.slot], cnt_t);
        atomicAdd(&a.counters[24 + a.slot], cnt_q);
        if (F32) atomicAdd(&a.counters[23], cnt_t);
    }
}

// One launch per slice of NIC components of the first ket shell, in the
// value type V of the work list.
template <int LA, int LB, int LC, int LD, int NIC, typename V, int IC0 = 0>
hipError_t launch_slices_v(const SRArgs &a, bool fold, hipStream_t st)
{
    if constexpr (IC0 >= ncart(LC)) {
        return hipSuccess;
    } else {
        const dim3 g((unsigned)std::max(1L, (a.max_entries + 255) / 256)), b(256);
        if (fold) hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD, V, true, IC0, NIC>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD, V, false, IC0, NIC>), g, b, 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_slices_v<LA, LB, LC, LD, NIC, V, IC0 + NIC>(a, fold, st);
    }
}

template <int LA, int LB, int LC, int LD, int NIC>
hipError_t launch_slices(const SRArgs &a, bool f32, bool fold, hipStream_t st)
{
    return f32 ? launch_slices_v<LA, LB, LC, LD, NIC, float>(a, fold, st)
               : launch_slices_v<LA, LB, LC, LD, NIC, double>(a, fold, st);
}

}  // namespace

}  // namespace pbcjk
