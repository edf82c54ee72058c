// Short-range J and K for the d class pairs whose contracted block does not
// fit in one lane's registers ((ss|dd) and total angular momentum L >= 5).
//
// One wavefront per group pair of the work list; the 64 lanes walk the
// primitive quartets and lattice shifts of the pair together (every
// screening decision is uniform across the wave):
//   - per shift, R^n_{tuv} level by level of the recurrence (Sec. 2.3, eq.
//     R_recursion), the values of one level spread over the lanes via LDS,
//     and summed over the shifts of the quartet (FP64, with the quartet's
//     prefactor) into Rs_{tuv};
//   - per quartet, the ket transform W[t][cd] += sum_s (-1)^{|s|} E^cd_s
//     Rs_{t+s}, accumulated over the ket primitives of the bra primitive;
//   - per bra primitive, the bra transform I[ab][cd] += sum_t E^ab_t W[t][cd],
//     each lane owning a fixed set of (ab, cd) entries in registers.
// At the end the block goes through LDS and every J/K target element is
// summed by one lane and added with one atomic.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_math.h"
#include "kernels.h"

namespace pbcjk {

namespace {

__host__ __device__ constexpr int nherm(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }

// Hermite index of (t,u,v), t+u+v <= L, in the order of increasing total
// degree, then t descending, then u descending.
__device__ __forceinline__ int hidx(int t, int u, int v)
{
    const int n = t + u + v;
    // entries of lower total degree: nherm(n-1); within degree n: (t, u) order
    const int base = n * (n + 1) * (n + 2) / 6;
    const int r = n - t;            // u + v
    return base + r * (r + 1) / 2 + (r - u);
}

template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(64) void k_sr_coop(SRArgs a)
{
    constexpr int L = LA + LB + LC + LD;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NAB = NA * NB, NCD = NC * ND;
    constexpr int LAB = LA + LB, LCD = LC + LD;
    constexpr int NH = nherm(L), NHAB = nherm(LAB);
    constexpr int NBLK = NAB * NCD, NW = NHAB * NCD;
    constexpr int PER = (NBLK + 63) / 64, PERW = (NW + 63) / 64, PERH = (NH + 63) / 64;
    constexpr int EB = (LA + 1) * (LB + 1) * (LAB + 1), EK = (LC + 1) * (LD + 1) * (LCD + 1);
    constexpr int NWB = (NBLK > NW) ? NBLK : NW;
    // the Boys lookups of a term are uniform over the wave: the table is read
    // from global memory (one broadcast load per coefficient)
    const double *tab = a.boys + L;
    __shared__ double sR[2][NH];
    __shared__ double sRs[NH];
    __shared__ double sW[NWB];        // W of one bra primitive; then the final block
    __shared__ double sEb[3][EB], sEk[3][EK];
    __shared__ int sT[NH][3];   // (t,u,v) of each Hermite index
    double *sBlk = sW;

    const int lane = threadIdx.x;
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v)
                if (lane == 0) { int h = hidx(t, u, v); sT[h][0] = t; sT[h][1] = u; sT[h][2] = v; }
    __syncthreads();
    const long count = (long)*a.count;
    unsigned long long cnt_q = 0, cnt_t = 0;

    for (long e = blockIdx.x; e < count; e += gridDim.x) {
    const int bi = a.nbr_bra[e], j = a.nbr_ket[e];
    const GroupRec gb = a.groups[a.gb0 + bi];
    const GroupRec gk = a.groups[a.gk0 + j];
    const int ns = a.nshell, n = a.nbfc;
    const int A = gb.shA, B = gb.shB, C = gk.shA, D = gk.shB;
    double wD = a.Dmax[A * ns + B];
    wD = fmax(wD, a.Dmax[C * ns + D]);
    wD = fmax(wD, a.Dmax[A * ns + C]);
    wD = fmax(wD, a.Dmax[A * ns + D]);
    wD = fmax(wD, a.Dmax[B * ns + C]);
    wD = fmax(wD, a.Dmax[B * ns + D]);
    // group-level density screen (already applied when the list was compacted)
    if (!(gb.Qmax * gk.Qmax * wD > a.d_schwarz)) continue;   // uniform over the wave

    double acc[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) acc[i] = 0.0;
    long ent_terms = 0;

    for (int pb = gb.pstart; pb < gb.pend; ++pb) {
        const PairRec Pb = a.pairs[pb];
        if (lane < 3) {
            EAxis<LA, LB> E;
            herm_axis<LA, LB>(0.5 / Pb.p, Pb.PA[lane], Pb.PB[lane], E);
            for (int i = 0; i <= LA; ++i)
                for (int jj = 0; jj <= LB; ++jj)
                    for (int t = 0; t <= LAB; ++t) sEb[lane][(i * (LB + 1) + jj) * (LAB + 1) + t] = E.v[i][jj][t];
        }
        double Wacc[PERW];
#pragma unroll
        for (int i = 0; i < PERW; ++i) Wacc[i] = 0.0;
        bool any_k = false;
        for (int pk = gk.pstart; pk < gk.pend; ++pk) {
            const PairRec Pk = a.pairs[pk];
            if (!(Pb.Q * Pk.Q * wD > a.d_schwarz)) continue;
            ++cnt_q;
            double rad2;
            if (!quartet_sphere(Pb, Pk, a.w2, a.d_ewald_R, rad2)) continue;
            const double p = Pb.p, q = Pk.p, pq = p * q;
            const double rho = pq / (p + q);
            double Rs[PERH];
#pragma unroll
            for (int i = 0; i < PERH; ++i) Rs[i] = 0.0;
            int nimg = 0;
            const double cen[3] = {Pb.P[0] - Pk.P[0], Pb.P[1] - Pk.P[1], Pb.P[2] - Pk.P[2]};
            for_images(a.lat, cen, rad2, a.rcap2, [&](const double *Lv, double L2) {
                ++nimg;
                double R0[L + 1];
                sr_R0<L, kBoysM>(rho, a.w2, L2, tab, a.bexp, R0);
                // R recurrence, one level at a time: level n holds t+u+v <= L-n
                int cur = 0;
                if (lane == 0) sR[0][0] = R0[L];
                __syncthreads();
                for (int lev = L - 1; lev >= 0; --lev) {
                    const int nv = nherm(L - lev), nxt = cur ^ 1;
                    for (int h = lane; h < nv; h += 64) {
                        const int t = sT[h][0], u = sT[h][1], v = sT[h][2];
                        double r;
                        if (h == 0) r = R0[lev];
                        else if (t > 0) r = (t >= 2 ? (t - 1) * sR[cur][hidx(t - 2, u, v)] : 0.0) + Lv[0] * sR[cur][hidx(t - 1, u, v)];
                        else if (u > 0) r = (u >= 2 ? (u - 1) * sR[cur][hidx(0, u - 2, v)] : 0.0) + Lv[1] * sR[cur][hidx(0, u - 1, v)];
                        else r = (v >= 2 ? (v - 1) * sR[cur][hidx(0, 0, v - 2)] : 0.0) + Lv[2] * sR[cur][hidx(0, 0, v - 1)];
                        sR[nxt][h] = r;
                    }
                    cur = nxt;
                    __syncthreads();
                }
#pragma unroll
                for (int i = 0; i < PERH; ++i) {
                    const int h = lane + 64 * i;
                    if (h < NH) Rs[i] += sR[cur][h];
                }
                __syncthreads();   // sR is rewritten by the next shift
            });
            if (nimg == 0) continue;
            cnt_t += nimg;
            ent_terms += nimg;
            any_k = true;
            const double pref = Pb.cpre * Pk.cpre * kTwoPi52 / (pq * sqrt(p + q));
#pragma unroll
            for (int i = 0; i < PERH; ++i) {
                const int h = lane + 64 * i;
                if (h < NH) sRs[h] = pref * Rs[i];
            }
            if (lane < 3) {
                EAxis<LC, LD> E;
                herm_axis<LC, LD>(0.5 / q, Pk.PA[lane], Pk.PB[lane], E);
                for (int i = 0; i <= LC; ++i)
                    for (int jj = 0; jj <= LD; ++jj)
                        for (int t = 0; t <= LCD; ++t) sEk[lane][(i * (LD + 1) + jj) * (LCD + 1) + t] = E.v[i][jj][t];
            }
            __syncthreads();
            // ket transform into the lane's W[t][cd] entries, t+u+v <= LAB
#pragma unroll
            for (int i = 0; i < PERW; ++i) {
                const int w = lane + 64 * i;
                if (w < NW) {
                    const int th = w / NCD, cd = w - th * NCD;
                    const int ic = cd / ND, id = cd - ic * ND;
                    const int t = sT[th][0], u = sT[th][1], v = sT[th][2];
                    const int ccx = cx(LC, ic), ccy = cy(LC, ic), ccz = cz(LC, ic);
                    const int dcx = cx(LD, id), dcy = cy(LD, id), dcz = cz(LD, id);
                    double s = 0.0;
                    for (int tt = 0; tt <= ccx + dcx; ++tt) {
                        const double ex = sEk[0][(ccx * (LD + 1) + dcx) * (LCD + 1) + tt];
                        for (int uu = 0; uu <= ccy + dcy; ++uu) {
                            const double ey = ex * sEk[1][(ccy * (LD + 1) + dcy) * (LCD + 1) + uu];
                            for (int vv = 0; vv <= ccz + dcz; ++vv) {
                                const double ez = ey * sEk[2][(ccz * (LD + 1) + dcz) * (LCD + 1) + vv];
                                const double rv = sRs[hidx(t + tt, u + uu, v + vv)];
                                s += ((tt + uu + vv) & 1) ? -ez * rv : ez * rv;
                            }
                        }
                    }
                    Wacc[i] += s;
                }
            }
            __syncthreads();   // sRs and sEk are rewritten by the next ket primitive
        }
        if (any_k) {
#pragma unroll
            for (int i = 0; i < PERW; ++i) {
                const int w = lane + 64 * i;
                if (w < NW) sW[w] = Wacc[i];
            }
            __syncthreads();
            // bra transform into the lane's block entries
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int k = lane + 64 * i;
                if (k < NBLK) {
                    const int ab = k / NCD, cd = k - ab * NCD;
                    const int ia = ab / NB, ib = ab - ia * NB;
                    const int acx = cx(LA, ia), acy = cy(LA, ia), acz = cz(LA, ia);
                    const int bcx = cx(LB, ib), bcy = cy(LB, ib), bcz = cz(LB, ib);
                    double s = 0.0;
                    for (int t = 0; t <= acx + bcx; ++t) {
                        const double ex = sEb[0][(acx * (LB + 1) + bcx) * (LAB + 1) + t];
                        for (int u = 0; u <= acy + bcy; ++u) {
                            const double ey = ex * sEb[1][(acy * (LB + 1) + bcy) * (LAB + 1) + u];
                            for (int v = 0; v <= acz + bcz; ++v)
                                s += ey * sEb[2][(acz * (LB + 1) + bcz) * (LAB + 1) + v] * sW[hidx(t, u, v) * NCD + cd];
                        }
                    }
                    acc[i] += s;
                }
            }
        }
        __syncthreads();   // sEb and sW are rewritten by the next bra primitive
    }
    if (ent_terms == 0) continue;   // uniform over the wave

    // contraction with the density through LDS
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int k = lane + 64 * i;
        if (k < NBLK) sBlk[k] = acc[i];
    }
    __syncthreads();
    const double w = (a.tri && j == bi) ? 0.5 : 1.0;
    const double *Dt = a.Dt;
    const int aoA = gb.aoA, aoB = gb.aoB, aoC = gk.aoA, aoD = gk.aoB;
    // targets: X[a,b] (NAB), X[c,d] (NCD), Y[a,c], Y[b,c], Y[a,d], Y[b,d]
    const int T0 = NAB, T1 = T0 + NCD, T2 = T1 + NA * NC, T3 = T2 + NB * NC, T4 = T3 + NA * ND, T5 = T4 + NB * ND;
    for (int t = lane; t < T5; t += 64) {
        double s = 0.0;
        if (t < T0) {
            const int ia = t / NB, ib = t - ia * NB;
            for (int ic = 0; ic < NC; ++ic)
                for (int id = 0; id < ND; ++id) s += sBlk[t * NCD + ic * ND + id] * Dt[(long)(aoC + ic) * n + aoD + id];
            atomicAdd(&a.X[(long)(aoA + ia) * n + aoB + ib], 2.0 * w * s);
        } else if (t < T1) {
            const int cd = t - T0, ic = cd / ND, id = cd - ic * ND;
            for (int ia = 0; ia < NA; ++ia)
                for (int ib = 0; ib < NB; ++ib) s += sBlk[(ia * NB + ib) * NCD + cd] * Dt[(long)(aoA + ia) * n + aoB + ib];
            atomicAdd(&a.X[(long)(aoC + ic) * n + aoD + id], 2.0 * w * s);
        } else if (t < T2) {
            const int r = t - T1, ia = r / NC, ic = r - ia * NC;
            for (int ib = 0; ib < NB; ++ib)
                for (int id = 0; id < ND; ++id)
                    s += sBlk[(ia * NB + ib) * NCD + ic * ND + id] * Dt[(long)(aoB + ib) * n + aoD + id];
            atomicAdd(&a.Y[(long)(aoA + ia) * n + aoC + ic], w * s);
        } else if (t < T3) {
            const int r = t - T2, ib = r / NC, ic = r - ib * NC;
            for (int ia = 0; ia < NA; ++ia)
                for (int id = 0; id < ND; ++id)
                    s += sBlk[(ia * NB + ib) * NCD + ic * ND + id] * Dt[(long)(aoA + ia) * n + aoD + id];
            atomicAdd(&a.Y[(long)(aoB + ib) * n + aoC + ic], w * s);
        } else if (t < T4) {
            const int r = t - T3, ia = r / ND, id = r - ia * ND;
            for (int ib = 0; ib < NB; ++ib)
                for (int ic = 0; ic < NC; ++ic)
                    s += sBlk[(ia * NB + ib) * NCD + ic * ND + id] * Dt[(long)(aoB + ib) * n + aoC + ic];
            atomicAdd(&a.Y[(long)(aoA + ia) * n + aoD + id], w * s);
        } else {
            const int r = t - T4, ib = r / ND, id = r - ib * ND;
            for (int ia = 0; ia < NA; ++ia)
                for (int ic = 0; ic < NC; ++ic)
                    s += sBlk[(ia * NB + ib) * NCD + ic * ND + id] * Dt[(long)(aoA + ia) * n + aoC + ic];
            atomicAdd(&a.Y[(long)(aoB + ib) * n + aoD + id], w * s);
        }
    }
    __syncthreads();   // sBlk is rewritten by the next entry
    }
    if (lane == 0) {
        atomicAdd(&a.counters[0], cnt_q);
        atomicAdd(&a.counters[1], cnt_t);
        atomicAdd(&a.counters[2 + a.slot], cnt_t);
        atomicAdd(&a.counters[24 + a.slot], cnt_q);
    }
}

// Up to total angular momentum 6, and groups of at most kCoopPrim primitive
// pairs: one wavefront per group pair, one primitive quartet per lane.
//   Phase A (lanes independent): screen, sphere, lattice shifts, the
//     recurrence in registers and Rs_{tuv} = pref sum_R1 R_{tuv} in FP64,
//     stored per lane in LDS;
//   Phase B (lanes together): for each quartet in order, W[t][cd] +=
//     sum_s (-1)^{|s|} E^cd_s Rs_{t+s} over lane-owned (t, cd); after the
//     last ket primitive of a bra primitive, I[ab][cd] += sum_t E^ab_t W[t][cd].
// The E coefficients of the group pair's primitive pairs are formed once in LDS.
constexpr int kCoopPrim = 9;

template <int L>
__host__ __device__ constexpr int coop_round() { return nherm(L) > 35 ? 32 : 64; }

template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(64) void k_sr_coop2(SRArgs a)
{
    constexpr int L = LA + LB + LC + LD;
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int NAB = NA * NB, NCD = NC * ND;
    constexpr int LAB = LA + LB, LCD = LC + LD;
    constexpr int NH = nherm(L), NHAB = nherm(LAB);
    constexpr int NBLK = NAB * NCD, NW = NHAB * NCD;
    constexpr int PER = (NBLK + 63) / 64, PERW = (NW + 63) / 64;
    constexpr int EB = (LA + 1) * (LB + 1) * (LAB + 1), EK = (LC + 1) * (LD + 1) * (LCD + 1);
    constexpr int NWB = (NBLK > NW) ? NBLK : NW;
    constexpr int QR = coop_round<L>();       // quartets per round
    const double *tab = a.boys + L;
    __shared__ double sRq[QR][NH];
    __shared__ double sEb[kCoopPrim][3][EB], sEk[kCoopPrim][3][EK];
    __shared__ double sW[NWB];
    __shared__ int sT[NH][3];
    __shared__ int sFlag[QR];
    double *sBlk = sW;

    const int lane = threadIdx.x;
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v)
                if (lane == 0) { int h = hidx(t, u, v); sT[h][0] = t; sT[h][1] = u; sT[h][2] = v; }
    __syncthreads();
    const long count = (long)*a.count;
    unsigned long long cnt_q = 0, cnt_t = 0;

    for (long e = blockIdx.x; e < count; e += gridDim.x) {
    const int bi = a.nbr_bra[e], j = a.nbr_ket[e];
    const GroupRec gb = a.groups[a.gb0 + bi];
    const GroupRec gk = a.groups[a.gk0 + j];
    const int ns = a.nshell, n = a.nbfc;
    const int A = gb.shA, B = gb.shB, C = gk.shA, D = gk.shB;
    double wD = a.Dmax[A * ns + B];
    wD = fmax(wD, a.Dmax[C * ns + D]);
    wD = fmax(wD, a.Dmax[A * ns + C]);
    wD = fmax(wD, a.Dmax[A * ns + D]);
    wD = fmax(wD, a.Dmax[B * ns + C]);
    wD = fmax(wD, a.Dmax[B * ns + D]);
    // group-level density screen (already applied when the list was compacted)
    if (!(gb.Qmax * gk.Qmax * wD > a.d_schwarz)) continue;   // uniform over the wave
    const int npb = gb.pend - gb.pstart, npk = gk.pend - gk.pstart, nq = npb * npk;

    // E coefficients of every primitive pair of the group pair
    for (int task = lane; task < 3 * (npb + npk); task += 64) {
        const int ax = task % 3, ip = task / 3;
        if (ip < npb) {
            const PairRec P = a.pairs[gb.pstart + ip];
            EAxis<LA, LB> E;
            herm_axis<LA, LB>(0.5 / P.p, P.PA[ax], P.PB[ax], E);
            for (int i = 0; i <= LA; ++i)
                for (int jj = 0; jj <= LB; ++jj)
                    for (int t = 0; t <= LAB; ++t) sEb[ip][ax][(i * (LB + 1) + jj) * (LAB + 1) + t] = E.v[i][jj][t];
        } else {
            const PairRec P = a.pairs[gk.pstart + ip - npb];
            EAxis<LC, LD> E;
            herm_axis<LC, LD>(0.5 / P.p, P.PA[ax], P.PB[ax], E);
            for (int i = 0; i <= LC; ++i)
                for (int jj = 0; jj <= LD; ++jj)
                    for (int t = 0; t <= LCD; ++t)
                        sEk[ip - npb][ax][(i * (LD + 1) + jj) * (LCD + 1) + t] = E.v[i][jj][t];
        }
    }
    __syncthreads();

    double acc[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) acc[i] = 0.0;
    double Wacc[PERW];
#pragma unroll
    for (int i = 0; i < PERW; ++i) Wacc[i] = 0.0;
    bool any_w = false;      // W of the current bra primitive has a term (uniform)
    long ent_terms = 0;      // uniform: summed over the wave below

    for (int q0 = 0; q0 < nq; q0 += QR) {
        // Phase A
        int flag = 0;
        if (lane < QR && q0 + lane < nq) {
            const int q = q0 + lane, ib = q / npk, ik = q - ib * npk;
            const PairRec Pb = a.pairs[gb.pstart + ib];
            const PairRec Pk = a.pairs[gk.pstart + ik];
            double rad2;
            if (Pb.Q * Pk.Q * wD > a.d_schwarz) {
                ++cnt_q;
                if (quartet_sphere(Pb, Pk, a.w2, a.d_ewald_R, rad2)) {
                    const double p = Pb.p, qq = Pk.p, pq = p * qq;
                    const double rho = pq / (p + qq);
                    const double cen[3] = {Pb.P[0] - Pk.P[0], Pb.P[1] - Pk.P[1], Pb.P[2] - Pk.P[2]};
                    double Rs[L + 1][L + 1][L + 1];
#pragma unroll
                    for (int t = 0; t <= L; ++t)
#pragma unroll
                        for (int u = 0; u <= L - t; ++u)
#pragma unroll
                            for (int v = 0; v <= L - t - u; ++v) Rs[t][u][v] = 0.0;
                    int nimg = 0;
                    for_images(a.lat, cen, rad2, a.rcap2, [&](const double *Lv, double L2) {
                        ++nimg;
                        double R0[L + 1];
                        sr_R0<L, kBoysM>(rho, a.w2, L2, tab, a.bexp, R0);
                        double R[L + 1][L + 1][L + 1];
                        herm_R<L, double>(R0, Lv[0], Lv[1], Lv[2], R);
#pragma unroll
                        for (int t = 0; t <= L; ++t)
#pragma unroll
                            for (int u = 0; u <= L - t; ++u)
#pragma unroll
                                for (int v = 0; v <= L - t - u; ++v) Rs[t][u][v] += R[t][u][v];
                    });
                    if (nimg) {
                        cnt_t += nimg;
                        flag = nimg;
                        const double pref = Pb.cpre * Pk.cpre * kTwoPi52 / (pq * sqrt(p + qq));
#pragma unroll
                        for (int t = 0; t <= L; ++t)
#pragma unroll
                            for (int u = 0; u <= L - t; ++u)
#pragma unroll
                                for (int v = 0; v <= L - t - u; ++v) sRq[lane][hidx(t, u, v)] = pref * Rs[t][u][v];
                    }
                }
            }
        }
        if (lane < QR) sFlag[lane] = flag;
        __syncthreads();
        // Phase B
        const int nr = (nq - q0) < QR ? (nq - q0) : QR;
        for (int jq = 0; jq < nr; ++jq) {
            const int q = q0 + jq, ib = q / npk, ik = q - ib * npk;
            if (sFlag[jq]) {
                ent_terms += sFlag[jq];
                any_w = true;
                const double *Rq = sRq[jq];
#pragma unroll
                for (int i = 0; i < PERW; ++i) {
                    const int w = lane + 64 * i;
                    if (w < NW) {
                        const int th = w / NCD, cd = w - th * NCD;
                        const int ic = cd / ND, id = cd - ic * ND;
                        const int t = sT[th][0], u = sT[th][1], v = sT[th][2];
                        const int ccx = cx(LC, ic), ccy = cy(LC, ic), ccz = cz(LC, ic);
                        const int dcx = cx(LD, id), dcy = cy(LD, id), dcz = cz(LD, id);
                        double s = 0.0;
                        for (int tt = 0; tt <= ccx + dcx; ++tt) {
                            const double ex = sEk[ik][0][(ccx * (LD + 1) + dcx) * (LCD + 1) + tt];
                            for (int uu = 0; uu <= ccy + dcy; ++uu) {
                                const double ey = ex * sEk[ik][1][(ccy * (LD + 1) + dcy) * (LCD + 1) + uu];
                                for (int vv = 0; vv <= ccz + dcz; ++vv) {
                                    const double ez = ey * sEk[ik][2][(ccz * (LD + 1) + dcz) * (LCD + 1) + vv];
                                    const double rv = Rq[hidx(t + tt, u + uu, v + vv)];
                                    s += ((tt + uu + vv) & 1) ? -ez * rv : ez * rv;
                                }
                            }
                        }
                        Wacc[i] += s;
                    }
                }
            }
            if (ik == npk - 1) {
                // last ket primitive of bra primitive ib: bra transform
                if (any_w) {
#pragma unroll
                    for (int i = 0; i < PERW; ++i) {
                        const int w = lane + 64 * i;
                        if (w < NW) sW[w] = Wacc[i];
                        Wacc[i] = 0.0;
                    }
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < PER; ++i) {
                        const int k = lane + 64 * i;
                        if (k < NBLK) {
                            const int ab = k / NCD, cd = k - ab * NCD;
                            const int ia = ab / NB, ibb = ab - ia * NB;
                            const int acx = cx(LA, ia), acy = cy(LA, ia), acz = cz(LA, ia);
                            const int bcx = cx(LB, ibb), bcy = cy(LB, ibb), bcz = cz(LB, ibb);
                            double s = 0.0;
                            for (int t = 0; t <= acx + bcx; ++t) {
                                const double ex = sEb[ib][0][(acx * (LB + 1) + bcx) * (LAB + 1) + t];
                                for (int u = 0; u <= acy + bcy; ++u) {
                                    const double ey = ex * sEb[ib][1][(acy * (LB + 1) + bcy) * (LAB + 1) + u];
                                    for (int v = 0; v <= acz + bcz; ++v)
                                        s += ey * sEb[ib][2][(acz * (LB + 1) + bcz) * (LAB + 1) + v] *
                                             sW[hidx(t, u, v) * NCD + cd];
                                }
                            }
                            acc[i] += s;
                        }
                    }
                    __syncthreads();
                    any_w = false;
                }
            }
        }
        __syncthreads();   // sRq and sFlag are rewritten by the next round
    }
    if (ent_terms == 0) continue;   // uniform over the wave

    // contraction with the density through LDS
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int k = lane + 64 * i;
        if (k < NBLK) sBlk[k] = acc[i];
    }
    __syncthreads();
    const double w = (a.tri && j == bi) ? 0.5 : 1.0;
    const double *Dt = a.Dt;
    const int aoA = gb.aoA, aoB = gb.aoB, aoC = gk.aoA, aoD = gk.aoB;
    const int T0 = NAB, T1 = T0 + NCD, T2 = T1 + NA * NC, T3 = T2 + NB * NC, T4 = T3 + NA * ND, T5 = T4 + NB * ND;
    for (int t = lane; t < T5; t += 64) {
        double s = 0.0;
        if (t < T0) {
            const int ia = t / NB, ib = t - ia * NB;
            for (int ic = 0; ic < NC; ++ic)
                for (int id = 0; id < ND; ++id) s += sBlk[t * NCD + ic * ND + id] * Dt[(long)(aoC + ic) * n + aoD + id];
            atomicAdd(&a.X[(long)(aoA + ia) * n + aoB + ib], 2.0 * w * s);
        } else if (t < T1) {
            const int cd = t - T0, ic = cd / ND, id = cd - ic * ND;
            for (int ia = 0; ia < NA; ++ia)
                for (int ib = 0; ib < NB; ++ib) s += sBlk[(ia * NB + ib) * NCD + cd] * Dt[(long)(aoA + ia) * n + aoB + ib];
            atomicAdd(&a.X[(long)(aoC + ic) * n + aoD + id], 2.0 * w * s);
        } else if (t < T2) {
            const int r = t - T1, ia = r / NC, ic = r - ia * NC;
            for (int ib = 0; ib < NB; ++ib)
                for (int id = 0; id < ND; ++id)
                    s += sBlk[(ia * NB + ib) * NCD + ic * ND + id] * Dt[(long)(aoB + ib) * n + aoD + id];
            atomicAdd(&a.Y[(long)(aoA + ia) * n + aoC + ic], w * s);
        } else if (t < T3) {
            const int r = t - T2, ib = r / NC, ic = r - ib * NC;
            for (int ia = 0; ia < NA; ++ia)
                for (int id = 0; id < ND; ++id)
                    s += sBlk[(ia * NB + ib) * NCD + ic * ND + id] * Dt[(long)(aoA + ia) * n + aoD + id];
            atomicAdd(&a.Y[(long)(aoB + ib) * n + aoC + ic], w * s);
        } else if (t < T4) {
            const int r = t - T3, ia = r / ND, id = r - ia * ND;
            for (int ib = 0; ib < NB; ++ib)
                for (int ic = 0; ic < NC; ++ic)
                    s += sBlk[(ia * NB + ib) * NCD + ic * ND + id] * Dt[(long)(aoB + ib) * n + aoC + ic];
            atomicAdd(&a.Y[(long)(aoA + ia) * n + aoD + id], w * s);
        } else {
            const int r = t - T4, ib = r / ND, id = r - ib * ND;
            for (int ia = 0; ia < NA; ++ia)
                for (int ic = 0; ic < NC; ++ic)
                    s += sBlk[(ia * NB + ib) * NCD + ic * ND + id] * Dt[(long)(aoA + ia) * n + aoC + ic];
            atomicAdd(&a.Y[(long)(aoB + ib) * n + aoD + id], w * s);
        }
    }
    __syncthreads();   // sBlk and the E coefficients are rewritten by the next entry
    }
    for (int off = 32; off > 0; off >>= 1) {
        cnt_q += __shfl_down(cnt_q, off, 64);
        cnt_t += __shfl_down(cnt_t, off, 64);
    }
    if (lane == 0) {
        atomicAdd(&a.counters[0], cnt_q);
        atomicAdd(&a.counters[1], cnt_t);
        atomicAdd(&a.counters[2 + a.slot], cnt_t);
        atomicAdd(&a.counters[24 + a.slot], cnt_q);
    }
}

template <int LA, int LB, int LC, int LD>
hipError_t launch_coop(const SRArgs &a, hipStream_t st)
{
    if (a.max_entries <= 0) return hipSuccess;
    const long grid = a.max_entries < 65536 ? a.max_entries : 65536;
    if constexpr (LA + LB + LC + LD <= 6) {
        if (a.max_prim_pairs <= kCoopPrim) {
            hipLaunchKernelGGL((k_sr_coop2<LA, LB, LC, LD>), dim3((unsigned)grid), dim3(64), 0, st, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_sr_coop<LA, LB, LC, LD>), dim3((unsigned)grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

constexpr int kLa[kNumClass] = {0, 1, 1, 2, 2, 2};
constexpr int kLb[kNumClass] = {0, 0, 1, 0, 1, 2};

}  // namespace

// d class pairs (cb <= ck) without a per-lane kernel.
hipError_t launch_sr_coop(int cb, int ck, const SRArgs &a, hipStream_t st)
{
#define PBCJK_CASE(X, Y) \
    if (cb == X && ck == Y) return launch_coop<kLa[X], kLb[X], kLa[Y], kLb[Y]>(a, st);
    PBCJK_CASE(0, 5) PBCJK_CASE(1, 5) PBCJK_CASE(2, 4) PBCJK_CASE(2, 5) PBCJK_CASE(3, 4) PBCJK_CASE(3, 5) PBCJK_CASE(4, 4)
    PBCJK_CASE(4, 5) PBCJK_CASE(5, 5)
#undef PBCJK_CASE
    return hipErrorNotSupported;
}

}  // namespace pbcjk
