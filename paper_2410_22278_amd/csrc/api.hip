// C ABI of the periodic J/K library (see include/pbcjk.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "arena.h"
#include "handle.h"
#include "kernels.h"
#include "pbcjk.h"

using namespace pbcjk;

namespace {

constexpr int kClassL[kNumClass] = {0, 1, 2, 2, 3, 4};
constexpr int kNumCounters = 48;     // see SRArgs::counters

// Large d class pairs with component-slice launches of the per-lane kernel.
bool sr_sliceable(int cb, int ck) { return !(cb == 5 && ck == 5); }

// Builds without K: class pairs whose bra is an s-s pair keep the fused J/K
// kernel, which is faster there than the J-engine (the Hermite densities of
// the bra would be loaded per quartet for a one-term contraction); the others
// run the J-engine.
bool sr_jengine(int cb, int ck) { return cb >= 1 && ck >= cb; }

// Class pairs (cb <= ck) with a per-lane register kernel: everything without
// a d shell, and the d pairs (ds|ss), (dp|ss), (ds|ps), (dp|ps), (ds|pp), (ds|ds).
bool sr_per_lane(int cb, int ck)
{
    if (cb < 3 && ck < 3) return true;
    const int lo = cb < ck ? cb : ck, hi = cb < ck ? ck : cb;
    return (lo == 0 && (hi == 3 || hi == 4)) || (lo == 1 && (hi == 3 || hi == 4)) || (lo == 2 && hi == 3) ||
           (lo == 3 && hi == 3);
}
constexpr double kFoldRmin = 20.0;   // bohr: cells with a shorter lattice vector start folded
constexpr double kFoldRatio = 1.1;   // shifts per quartet above which the lattice sum is folded
constexpr long kStage2Blocks = 4096; // workgroups aimed at by the split exchange accumulation
constexpr double kCoopRatio = 4.5;   // shifts per quartet above which large d pairs use one
                                     // wavefront per group pair (it evaluates each shift once)
constexpr int kFp32MinL = 4;         // mixed precision: class pairs of at least this total angular
                                     // momentum run their low-bound group pairs in FP32

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

}  // namespace

// Sets the thread's last-error message (other translation units of the library).
int pbcjk::set_error(int code, const char *msg) { return fail(code, msg ? msg : ""); }

namespace {

#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(PBC_JK_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

struct pbc_jk {
    Setup S;
    int device = 0;
    Arena *arena = nullptr;      // device memory source; NULL = hipMalloc
    size_t dev_bytes = 0;        // device bytes held
    bool profile = true;         // per-launch timing events (GEMM, structure factors)
    double lr_budget_mb = 0.0;   // reciprocal chunk budget; 0 = default
    bool dry = false;            // count device bytes only (no allocation, no copies)
    size_t dry_bytes = 0;
    int parts = PBC_JK_PART_SR | PBC_JK_PART_LR | PBC_JK_PART_SELF;
    int lr_mode = PBC_JK_LR_AUTO;
    int sr_classes = (1 << 21) - 1;
    double lr_tol = 1e-13;
    hipStream_t own = nullptr;
    // setup data
    PairRec *d_pairs = nullptr;
    GroupRec *d_groups = nullptr;
    double *d_boys = nullptr, *d_bexp = nullptr, *d_S = nullptr, *d_G = nullptr, *d_Gw = nullptr, *d_Gs = nullptr;
    int *d_sp_start = nullptr, *d_sp_pairs = nullptr, *d_sp_shA = nullptr, *d_sp_shB = nullptr;
    int *d_sh_l = nullptr, *d_sh_aoc = nullptr, *d_tr_ao = nullptr, *d_inv_ci = nullptr;
    double *d_tr_c = nullptr, *d_dscale = nullptr, *d_inv_cc = nullptr;
    // build work space
    double *d_D = nullptr, *d_Dt = nullptr, *d_Dmax = nullptr, *d_X = nullptr, *d_Y = nullptr;
    double *d_Jt = nullptr, *d_Kt = nullptr, *d_F = nullptr, *d_T = nullptr, *d_rho = nullptr;
    // The structure-factor kernels overwrite every block of the shell pairs
    // in the pair list and nothing else writes F, so once the handle's own F
    // has been cleared the blocks of absent shell pairs stay zero: f_clean is
    // the buffer known to be in that state (a buffer lent by the static
    // entry point is cleared at every use).
    const double *f_clean = nullptr, *f_own = nullptr;
    double *d_scal = nullptr, *d_Jo = nullptr, *d_Ko = nullptr;
    unsigned long long *d_dmaxg = nullptr, *d_cnt = nullptr;
    unsigned long long *stat_cnt = nullptr;   // counters of the last build (own or scratch buffer)
    // J-engine: Hermite densities of every primitive pair (per class, pairs
    // p0 .. of the class at hd + hd_base[class])
    double *d_hd = nullptr;
    double *d_xyz = nullptr, *d_q = nullptr;   // atom positions, point charges -Z (one-electron terms)
    long hd_base[kNumClass + 1] = {0};
    int class_p0[kNumClass] = {0};
    // real-space neighbour lists, one segment per class pair
    int *d_nbr_bra = nullptr, *d_nbr_ket = nullptr;
    // low-rank reciprocal exchange: density factor (by columns), work, control
    double *d_L = nullptr, *d_pw = nullptr;
    int *d_pwi = nullptr, *d_ctl = nullptr;
    int *h_ctl = nullptr;        // pinned copy of the control block of the last finished factor
    hipEvent_t ev_ctl = nullptr; // recorded after that copy
    int lr_cap = 0;              // columns queued for the last factor (upper bound of its rank)
    int y_tile = 64;             // output tile of the products Y_b^T = L^T F_b
    // stream capture of the host-memory build: the device work of one build
    // (D in d_D to J, K in d_Jo, d_Ko and the energies in d_scal) as a graph
    bool use_graph = false, capturing = false;
    // whether the last build's counters and factor decision were readable when
    // the capture began (no event query runs inside a capture)
    bool cnt_done = false, ctl_done = false;
    hipGraphExec_t gexec = nullptr;
    double coop_ratio = kCoopRatio;
    int fp32_min_l = kFp32MinL;
    bool chol_panel = true;        // blocked density factor (else one launch per column)
    bool serial_lr = false;        // reciprocal part after the short range (else concurrently)
    bool y_tall = true;            // low-rank products in 512-row panels (k_ygemm) when the reciprocal
                                   // part runs alone, else k_dgemm<2>
    bool y_always = false;         // k_ygemm beside the short range too
    bool factor_first = true;      // density factor on the build stream before the short range
    int lr_rmax = 0;
    bool lr_ran = false;
    size_t nbr_bytes_needed = 0;   // set once the neighbour lists are counted
    long nbr_off[22] = {0};
    // per-build work lists (density-screened neighbour lists, FP64 and FP32)
    // at the same offsets, and their lengths (2 per class pair)
    int *d_w64b = nullptr, *d_w64k = nullptr, *d_w32b = nullptr, *d_w32k = nullptr;
    unsigned long long *d_wcnt = nullptr;
    long long *d_pcc = nullptr;   // chunk counts of the order-preserving FP64/FP32 split
    unsigned long long *d_ncnt = nullptr;   // neighbour-list segment lengths (21)
    // counters of the last finished build (pinned copy, event-guarded), used
    // to choose per class pair whether the lattice sum is folded into R_{tuv}
    unsigned long long *h_cnt = nullptr;
    hipEvent_t ev_cnt = nullptr;
    bool fold[21] = {false};
    int class_max_pp[6] = {0};   // most primitive pairs in one group, per class
    bool coop_d[21] = {false};   // large d class pairs: one wavefront per group pair (else slices)
    int gchunk = 0;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // the reciprocal part and the self term run on `side`, beside the short
    // range on the build stream: fork after the density preparation, join
    // before the final assembly
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the first reciprocal chunk's structure factors and J run on `side2`
    // while `side` factorises the density
    hipStream_t side2 = nullptr;
    hipEvent_t ev_sf = nullptr;
    // event pairs around GEMM and structure-factor launches of one build
    static constexpr int kMaxTimed = 4096;
    std::vector<hipEvent_t> tev;
    // 0 = plain GEMM (k_dgemm<0>), 1 = structure factors, 2 = residual check
    // of the density factor (k_dgemm<1>), 4 = factorisation, 5 + slot = the
    // short-range launch of class pair `slot` (5..25), 30 = Y_b^T = L^T F_b
    // (k_dgemm<2>), 31 = K += sum_b Y_b Y_b^T (k_dgemm<3>); for 30 and 31 the
    // recorded FLOPs are per unit of the density rank
    std::vector<int> tkind;
    std::vector<double> tflops;
    int ntimed = 0;
    bool timed = false;
    pbc_jk_counters st{};
};

namespace {

template <class T>
int dalloc(pbc_jk *h, T **p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    const size_t bytes = n * sizeof(T);
    if (h->dry) {
        h->dry_bytes += Arena::round_up(bytes);
        return 0;
    }
    if (h->arena) {
        *p = (T *)h->arena->alloc(bytes);
        if (!*p) return fail(PBC_JK_ENOMEM, "device memory budget exhausted");
        h->dev_bytes += Arena::round_up(bytes);
        return 0;
    }
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(PBC_JK_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    h->dev_bytes += bytes;
    return 0;
}

void dfree(pbc_jk *h, void *p)
{
    if (!p) return;
    if (h->arena && h->arena->owns(p)) {
        h->arena->release(p);
        return;
    }
    (void)hipFree(p);
}

template <class T>
int upload(pbc_jk *h, T **p, const std::vector<T> &v)
{
    int rc = dalloc(h, p, v.size());
    if (rc || h->dry) return rc;
    if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return 0;
}

// Frees the device buffers (pointers reset; streams, events and the host
// setup are kept, so the device part can be created again).
void release_device(pbc_jk *h)
{
    void **pp[] = {(void **)&h->d_pairs, (void **)&h->d_groups, (void **)&h->d_boys, (void **)&h->d_bexp, (void **)&h->d_S,
                   (void **)&h->d_G, (void **)&h->d_Gw, (void **)&h->d_Gs,
                   (void **)&h->d_sp_start, (void **)&h->d_sp_pairs,
                   (void **)&h->d_sp_shA, (void **)&h->d_sp_shB, (void **)&h->d_sh_l, (void **)&h->d_sh_aoc,
                   (void **)&h->d_tr_ao, (void **)&h->d_inv_ci, (void **)&h->d_tr_c, (void **)&h->d_dscale,
                   (void **)&h->d_inv_cc, (void **)&h->d_D, (void **)&h->d_Dt, (void **)&h->d_Dmax,
                   (void **)&h->d_X, (void **)&h->d_Y, (void **)&h->d_Jt, (void **)&h->d_Kt, (void **)&h->d_F,
                   (void **)&h->d_T, (void **)&h->d_rho, (void **)&h->d_scal, (void **)&h->d_Jo,
                   (void **)&h->d_Ko, (void **)&h->d_dmaxg, (void **)&h->d_cnt, (void **)&h->d_nbr_bra,
                   (void **)&h->d_nbr_ket, (void **)&h->d_L, (void **)&h->d_pw, (void **)&h->d_pwi,
                   (void **)&h->d_ctl, (void **)&h->d_w64b, (void **)&h->d_w64k, (void **)&h->d_w32b,
                   (void **)&h->d_w32k, (void **)&h->d_wcnt, (void **)&h->d_pcc, (void **)&h->d_ncnt,
                   (void **)&h->d_hd, (void **)&h->d_xyz, (void **)&h->d_q};
    for (void **p : pp) {
        dfree(h, *p);
        *p = nullptr;
    }
    h->dev_bytes = 0;
    h->timed = false;
    h->f_clean = h->f_own = nullptr;
}

void drop_graph(pbc_jk *h);

void release(pbc_jk *h)
{
    drop_graph(h);
    release_device(h);
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : h->tev)
        if (e) (void)hipEventDestroy(e);
    if (h->ev_cnt) (void)hipEventDestroy(h->ev_cnt);
    h->ev_cnt = nullptr;
    if (h->ev_ctl) (void)hipEventDestroy(h->ev_ctl);
    h->ev_ctl = nullptr;
    if (h->h_cnt) (void)hipHostFree(h->h_cnt);
    h->h_cnt = nullptr;
    if (h->h_ctl) (void)hipHostFree(h->h_ctl);
    h->h_ctl = nullptr;
    if (h->own) (void)hipStreamDestroy(h->own);
    h->own = nullptr;
    if (h->side) (void)hipStreamDestroy(h->side);
    h->side = nullptr;
    if (h->side2) (void)hipStreamDestroy(h->side2);
    h->side2 = nullptr;
    if (h->ev_sf) (void)hipEventDestroy(h->ev_sf);
    h->ev_sf = nullptr;
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    h->ev_fork = h->ev_join = nullptr;
    for (auto &e : h->ev) e = nullptr;
    h->tev.clear();
}

// Brackets one launch with a pair of events (up to kMaxTimed per build).
struct TimedLaunch {
    pbc_jk *h;
    hipStream_t st;
    int slot = -1;
    TimedLaunch(pbc_jk *h_, hipStream_t st_, int kind, double flops) : h(h_), st(st_)
    {
        if (h->profile && !h->capturing && h->ntimed < pbc_jk::kMaxTimed) {
            slot = h->ntimed++;
            h->tkind[slot] = kind;
            h->tflops[slot] = flops;
            (void)hipEventRecord(h->tev[2 * slot], st);
        }
    }
    ~TimedLaunch()
    {
        if (slot >= 0) (void)hipEventRecord(h->tev[2 * slot + 1], st);
    }
};

int build_neighbours(pbc_jk *h);

int create_device(pbc_jk *h)
{
    Setup &S = h->S;
    if (!h->dry) {
        HIPCHK(hipGetDevice(&h->device));
        if (!h->own) HIPCHK(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking));
        if (!h->side) HIPCHK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        if (!h->side2) HIPCHK(hipStreamCreateWithFlags(&h->side2, hipStreamNonBlocking));
        if (!h->ev_sf) HIPCHK(hipEventCreateWithFlags(&h->ev_sf, hipEventDisableTiming));
        if (!h->ev_fork) HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        if (!h->ev_join) HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
        for (auto &e : h->ev)
            if (!e) HIPCHK(hipEventCreate(&e));
        if (h->profile && h->tev.empty()) {
            h->tev.assign(2 * pbc_jk::kMaxTimed, nullptr);
            h->tkind.assign(pbc_jk::kMaxTimed, 0);
            h->tflops.assign(pbc_jk::kMaxTimed, 0.0);
            for (auto &e : h->tev) HIPCHK(hipEventCreate(&e));
        }
    }
    int rc;
    if ((rc = upload(h, &h->d_pairs, S.pairs))) return rc;
    if ((rc = upload(h, &h->d_groups, S.groups))) return rc;
    if ((rc = upload(h, &h->d_boys, S.boys))) return rc;
    if ((rc = upload(h, &h->d_bexp, S.bexp))) return rc;
    if ((rc = upload(h, &h->d_S, S.S))) return rc;
    if ((rc = upload(h, &h->d_G, S.G))) return rc;
    if ((rc = upload(h, &h->d_Gw, S.Gw))) return rc;
    if ((rc = upload(h, &h->d_Gs, S.Gs))) return rc;
    if ((rc = upload(h, &h->d_sp_start, S.sp_start))) return rc;
    if ((rc = upload(h, &h->d_sp_pairs, S.sp_pairs))) return rc;
    if ((rc = upload(h, &h->d_sp_shA, S.sp_shA))) return rc;
    if ((rc = upload(h, &h->d_sp_shB, S.sp_shB))) return rc;
    if ((rc = upload(h, &h->d_sh_l, S.sh_l))) return rc;
    if ((rc = upload(h, &h->d_sh_aoc, S.sh_aoc))) return rc;
    if ((rc = upload(h, &h->d_tr_ao, S.tr_ao))) return rc;
    if ((rc = upload(h, &h->d_tr_c, S.tr_c))) return rc;
    if ((rc = upload(h, &h->d_dscale, S.dscale))) return rc;
    if ((rc = upload(h, &h->d_xyz, S.xyz))) return rc;
    {
        std::vector<double> q(S.natom, 0.0);
        for (size_t i = 0; i < S.charge.size(); ++i) q[i] = -S.charge[i];
        if ((rc = upload(h, &h->d_q, q))) return rc;
    }
    // inverse transform: output AO -> up to three (Cartesian index, coefficient)
    std::vector<int> ici(3 * S.nbf, -1);
    std::vector<double> icc(3 * S.nbf, 0.0);
    std::vector<int> fillc(S.nbf, 0);
    for (int i = 0; i < S.nbfc; ++i)
        for (int u = 0; u < 2; ++u) {
            int a = S.tr_ao[2 * i + u];
            if (a < 0) continue;
            int k = fillc[a]++;
            if (k >= 3) return fail(PBC_JK_EINVAL, "internal: transform fan-in above 3");
            ici[3 * a + k] = i;
            icc[3 * a + k] = S.tr_c[2 * i + u];
        }
    if ((rc = upload(h, &h->d_inv_ci, ici))) return rc;
    if ((rc = upload(h, &h->d_inv_cc, icc))) return rc;

    const size_t n2 = (size_t)S.nbfc * S.nbfc, m2 = (size_t)S.nbf * S.nbf;
    if ((rc = dalloc(h, &h->d_D, m2))) return rc;
    if ((rc = dalloc(h, &h->d_Dt, n2))) return rc;
    if ((rc = dalloc(h, &h->d_Dmax, (size_t)S.nshell * S.nshell))) return rc;
    if ((rc = dalloc(h, &h->d_X, n2))) return rc;
    if ((rc = dalloc(h, &h->d_Y, n2))) return rc;
    if ((rc = dalloc(h, &h->d_Jt, n2))) return rc;
    if ((rc = dalloc(h, &h->d_Kt, n2))) return rc;
    if ((rc = dalloc(h, &h->d_Jo, m2))) return rc;
    if ((rc = dalloc(h, &h->d_Ko, m2))) return rc;
    if ((rc = dalloc(h, &h->d_scal, 4))) return rc;
    if ((rc = dalloc(h, &h->d_dmaxg, 1))) return rc;
    if ((rc = dalloc(h, &h->d_cnt, kNumCounters))) return rc;
    for (int c = 0; c < kNumClass; ++c) {
        h->class_max_pp[c] = 0;
        for (int g = S.class_start[c]; g < S.class_start[c + 1]; ++g)
            h->class_max_pp[c] = std::max(h->class_max_pp[c], S.groups[g].pend - S.groups[g].pstart);
    }
    // Hermite densities: n_h(l_a + l_b) values per pair, class by class (the
    // pairs of a class are contiguous, in the order of its groups)
    h->hd_base[0] = 0;
    for (int c = 0; c < kNumClass; ++c) {
        const int g0 = S.class_start[c], g1 = S.class_start[c + 1];
        const int p0 = g0 < g1 ? S.groups[g0].pstart : 0, p1 = g0 < g1 ? S.groups[g1 - 1].pend : 0;
        const int lab = kClassL[c];
        h->class_p0[c] = p0;
        h->hd_base[c + 1] = h->hd_base[c] + (long)(p1 - p0) * ((lab + 1) * (lab + 2) * (lab + 3) / 6);
    }
    if ((rc = dalloc(h, &h->d_hd, (size_t)std::max(1L, h->hd_base[kNumClass])))) return rc;
    if (!h->dry) {
        if (!h->h_cnt) HIPCHK(hipHostMalloc((void **)&h->h_cnt, kNumCounters * sizeof(unsigned long long)));
        if (!h->h_ctl) HIPCHK(hipHostMalloc((void **)&h->h_ctl, 4 * sizeof(int)));
        std::memset(h->h_ctl, 0, 4 * sizeof(int));
        std::memset(h->h_cnt, 0, kNumCounters * sizeof(unsigned long long));
        if (!h->ev_cnt) HIPCHK(hipEventCreateWithFlags(&h->ev_cnt, hipEventDisableTiming));
        if (!h->ev_ctl) HIPCHK(hipEventCreateWithFlags(&h->ev_ctl, hipEventDisableTiming));
        // first guess: quartets of small cells have several lattice shifts
        for (bool &f : h->fold) f = S.lat.Rmin < kFoldRmin;
    }
    // reciprocal-space chunk: F and T hold 2 * gchunk matrices each
    if (const char *e = std::getenv("PBCJK_Y_TILE")) h->y_tile = std::atoi(e) == 128 ? 128 : 64;
    if (const char *e = std::getenv("PBCJK_COOP_RATIO")) h->coop_ratio = std::max(0.0, std::atof(e));
    if (const char *e = std::getenv("PBCJK_FP32_MIN_L")) h->fp32_min_l = std::max(0, std::atoi(e));
    if (const char *e = std::getenv("PBCJK_CHOL_PANEL")) h->chol_panel = std::atoi(e) != 0;
    if (const char *e = std::getenv("PBCJK_SERIAL_LR")) h->serial_lr = std::atoi(e) != 0;
    if (const char *e = std::getenv("PBCJK_YGEMM")) h->y_tall = std::atoi(e) != 0;
    if (const char *e = std::getenv("PBCJK_YGEMM_ALWAYS")) h->y_always = std::atoi(e) != 0;
    if (const char *e = std::getenv("PBCJK_FACTOR_FIRST")) h->factor_first = std::atoi(e) != 0;
    const int nG = (int)S.Gw.size();
    double budget_mb = h->lr_budget_mb > 0 ? h->lr_budget_mb : 16384.0;
    if (const char *e = std::getenv("PBCJK_LR_BUDGET_MB")) budget_mb = std::max(64.0, std::atof(e));
    long per = (long)(budget_mb * 1048576.0 / (4.0 * 8.0 * (double)n2));
    h->gchunk = (int)std::max(1L, std::min<long>(per, std::max(nG, 1)));
    if ((rc = dalloc(h, &h->d_F, 2 * (size_t)h->gchunk * n2))) return rc;
    h->f_own = h->d_F;
    h->f_clean = nullptr;
    if ((rc = dalloc(h, &h->d_T, std::max<size_t>(2 * (size_t)h->gchunk * n2, n2)))) return rc;
    if ((rc = dalloc(h, &h->d_rho, 2 * (size_t)h->gchunk))) return rc;
    const int n = S.nbfc, nblk = (n + 63) / 64;
    h->lr_rmax = std::max(1, (3 * n) / 4);
    if ((rc = dalloc(h, &h->d_L, (size_t)n * h->lr_rmax))) return rc;
    if ((rc = dalloc(h, &h->d_pw, (size_t)n + 2 * nblk + 4))) return rc;
    if ((rc = dalloc(h, &h->d_pwi, 2 * (size_t)nblk))) return rc;
    if ((rc = dalloc(h, &h->d_ctl, 4))) return rc;
    if (h->dry) return 0;
    return build_neighbours(h);
}

LatArgs lat_args(const Setup &S)
{
    LatArgs l;
    std::memcpy(l.M, S.lat.M, sizeof l.M);
    std::memcpy(l.Minv, S.lat.Minv, sizeof l.Minv);
    std::memcpy(l.span, S.lat.span, sizeof l.span);
    l.Rmin = S.lat.Rmin;
    return l;
}

// Width of the distance buckets of the neighbour lists (bohr).
constexpr double kNbrBucketWidth = 2.0;

// Real-space neighbour lists of every class pair: count per (bra group,
// distance bucket), scan on the host, fill in bra order, nearest buckets
// first inside each bra group.
int build_neighbours(pbc_jk *h)
{
    const Setup &S = h->S;
    hipStream_t st = h->own;
    NbrArgs a{};
    a.pairs = h->d_pairs; a.groups = h->d_groups; a.lat = lat_args(S);
    a.w2 = S.omega * S.omega; a.d_ewald_R = S.d_ewald_R; a.rcap2 = S.r_cut > 0 ? S.r_cut * S.r_cut : 0.0;
    double bw = kNbrBucketWidth;
    if (const char *e = std::getenv("PBCJK_NBR_BW")) bw = std::atof(e);
    a.inv_bw = bw > 0 ? 1.0 / bw : 0.0;
    int maxnb = 0;
    for (int c = 0; c < kNumClass; ++c) maxnb = std::max(maxnb, S.class_start[c + 1] - S.class_start[c]);
    const long maxnc = (long)std::max(1, maxnb) * kNbrBuckets;
    int *d_counts = nullptr;
    long *d_offs = nullptr;
    int rc;
    struct Tmp {
        pbc_jk *h;
        void *a = nullptr, *b = nullptr;
        ~Tmp() { dfree(h, a); dfree(h, b); }
    } tmp{h};
    if ((rc = dalloc(h, &d_counts, maxnc))) return rc;
    tmp.a = d_counts;
    if ((rc = dalloc(h, &d_offs, maxnc))) return rc;
    tmp.b = d_offs;
    // per class pair: the (bra group, bucket) counts, scanned when written
    std::vector<std::vector<int>> cnts(21);
    std::vector<long> offs(maxnc);
    long total = 0;
    int slot = 0;
    for (int cb = 0; cb < kNumClass; ++cb)
        for (int ck = cb; ck < kNumClass; ++ck, ++slot) {
            h->nbr_off[slot] = total;
            a.gb0 = S.class_start[cb]; a.nb = S.class_start[cb + 1] - S.class_start[cb];
            a.gk0 = S.class_start[ck]; a.nk = S.class_start[ck + 1] - S.class_start[ck];
            a.tri = (cb == ck);
            if (a.nb == 0 || a.nk == 0) continue;
            a.mode = 0; a.counts = d_counts;
            HIPCHK(launch_nbr(a, st));
            const long nc = (long)a.nb * kNbrBuckets;
            cnts[slot].resize(nc);
            HIPCHK(hipMemcpyAsync(cnts[slot].data(), d_counts, nc * sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (long i = 0; i < nc; ++i) total += cnts[slot][i];
        }
    h->nbr_off[21] = total;
    // the FP64/FP32 work lists exist only with mixed precision
    const size_t ne = (size_t)std::max(1L, total), nw = S.fp32_below > 0 ? ne : 1;
    long max_chunks = 1;
    for (int k = 0; k < 21; ++k)
        max_chunks = std::max(max_chunks, (h->nbr_off[k + 1] - h->nbr_off[k] + kPartChunk - 1) / kPartChunk);
    const size_t npcc = S.fp32_below > 0 ? 2 * (size_t)max_chunks : 2;
    h->nbr_bytes_needed = 2 * Arena::round_up(sizeof(int) * ne) + 4 * Arena::round_up(sizeof(int) * nw) +
                          Arena::round_up(42 * sizeof(unsigned long long)) +
                          Arena::round_up(21 * sizeof(unsigned long long)) +
                          Arena::round_up(npcc * sizeof(long long));
    if ((rc = dalloc(h, &h->d_nbr_bra, ne)) || (rc = dalloc(h, &h->d_nbr_ket, ne)) ||
        (rc = dalloc(h, &h->d_w64b, nw)) || (rc = dalloc(h, &h->d_w64k, nw)) ||
        (rc = dalloc(h, &h->d_w32b, nw)) || (rc = dalloc(h, &h->d_w32k, nw)) ||
        (rc = dalloc(h, &h->d_wcnt, 42)) || (rc = dalloc(h, &h->d_ncnt, 21)) ||
        (rc = dalloc(h, &h->d_pcc, npcc)))
        return rc;
    slot = 0;
    for (int cb = 0; cb < kNumClass; ++cb)
        for (int ck = cb; ck < kNumClass; ++ck, ++slot) {
            a.gb0 = S.class_start[cb]; a.nb = S.class_start[cb + 1] - S.class_start[cb];
            a.gk0 = S.class_start[ck]; a.nk = S.class_start[ck + 1] - S.class_start[ck];
            a.tri = (cb == ck);
            if (a.nb == 0 || a.nk == 0 || h->nbr_off[slot + 1] == h->nbr_off[slot]) continue;
            const long nc = (long)a.nb * kNbrBuckets;
            long pos = h->nbr_off[slot];
            for (long i = 0; i < nc; ++i) { offs[i] = pos; pos += cnts[slot][i]; }
            std::vector<int>().swap(cnts[slot]);
            HIPCHK(hipMemcpyAsync(d_offs, offs.data(), nc * sizeof(long), hipMemcpyHostToDevice, st));
            a.mode = 1; a.offsets = d_offs; a.out_bra = h->d_nbr_bra; a.out_ket = h->d_nbr_ket;
            HIPCHK(launch_nbr(a, st));
            HIPCHK(hipStreamSynchronize(st));
        }
    h->st.n_group_pairs = (double)total;
    unsigned long long seg[21];
    for (int k = 0; k < 21; ++k) seg[k] = (unsigned long long)(h->nbr_off[k + 1] - h->nbr_off[k]);
    HIPCHK(hipMemcpy(h->d_ncnt, seg, sizeof seg, hipMemcpyHostToDevice));
    return 0;
}

// An event that has completed; a pending one leaves no error behind for the
// launch checks that follow.
bool event_done(hipEvent_t e)
{
    if (!e) return false;
    const hipError_t q = hipEventQuery(e);
    if (q != hipSuccess) (void)hipGetLastError();
    return q == hipSuccess;
}

int run_build_streams(pbc_jk *h, const double *dD, double *dJ, double *dK, double *E_J, double *E_K, hipStream_t st)
{
    Setup &S = h->S;
    const int n = S.nbfc, nb = S.nbf;
    const long n2 = (long)n * n, m2 = (long)nb * nb;
    const bool wantJ = dJ || E_J, wantK = dK || E_K;
    double *Jo = dJ ? dJ : h->d_Jo;
    double *Ko = dK ? dK : h->d_Ko;
    h->ntimed = 0;
    h->stat_cnt = h->d_cnt;
    if (!h->capturing) HIPCHK(hipEventRecord(h->ev[0], st));

    // B1: density in the scaled Cartesian basis, block maxima
    HIPCHK(launch_fill((double *)h->d_dmaxg, 1, 0.0, st));
    DprepArgs dp{dD, nb, n, S.nshell, h->d_tr_ao, h->d_tr_c, h->d_dscale, h->d_sh_aoc, h->d_sh_l,
                 h->d_Dt, h->d_Dmax, h->d_dmaxg};
    HIPCHK(launch_dprep(dp, st));
    HIPCHK(launch_fill(h->d_X, n2, 0.0, st));
    HIPCHK(launch_fill(h->d_Y, n2, 0.0, st));
    HIPCHK(launch_fill(h->d_Jt, n2, 0.0, st));
    HIPCHK(launch_fill(h->d_Kt, n2, 0.0, st));
    HIPCHK(launch_fill((double *)h->d_cnt, kNumCounters, 0.0, st));
    // class pairs whose quartets had several shifts each in the last finished
    // build sum the shifts before the transforms
    if (h->capturing ? h->cnt_done : event_done(h->ev_cnt))
        for (int k = 0; k < 21; ++k) {
            const double nq = (double)h->h_cnt[24 + k], nt = (double)h->h_cnt[2 + k];
            if (nq > 0) {
                h->fold[k] = nt > kFoldRatio * nq;
                h->coop_d[k] = nt > h->coop_ratio * nq;
            }
        }

    // B6 prelude: the density factor of the low-rank exchange, whose rank
    // stays on the device.  By default it runs on the build stream before the
    // short range (its column steps are short launches that the short-range
    // kernels would hold back); the reciprocal products wait for it.
    const int nG = (int)S.Gw.size();
    const bool lr_on = (h->parts & PBC_JK_PART_LR) && nG > 0 && (wantJ || wantK);
    const bool lowrank = lr_on && wantK && h->lr_mode == PBC_JK_LR_AUTO;
    h->lr_ran = lowrank;
    // Columns queued for the density factor: the rank of the last finished
    // factor plus a margin when it is known without waiting, else the limit.
    // A factor that needs more columns than queued does not converge and the
    // dense form runs instead (decided on the device); the next build then
    // queues the limit again.
    int cap = h->lr_rmax;
    if (lowrank && (h->capturing ? h->ctl_done : event_done(h->ev_ctl)) && h->h_ctl[2] && !h->h_ctl[1] &&
        h->h_ctl[0] > 0)
        cap = std::min(h->lr_rmax, ((h->h_ctl[0] + 64 + 63) / 64) * 64);
    auto run_factor = [&](hipStream_t s) -> int {
        // D~ = L L^T on the device; R = L L^T into T, then the entrywise check.
        // The rank and the choice of form stay in the control block: every
        // product below reads them there, so nothing waits on the host.
        {
            TimedLaunch tl(h, s, 4, 0.0);
            HIPCHK(launch_pchol(h->d_Dt, n, h->lr_tol, cap, h->d_L, h->d_pw, h->d_pwi, h->d_ctl,
                                h->chol_panel ? h->d_T : nullptr, s));
        }
        GemmArgs gr{};
        gr.M = gr.N = n; gr.K = cap;
        gr.A = h->d_L; gr.lda = n; gr.sA = 0; gr.transA = 1;
        gr.B = h->d_L; gr.ldb = n; gr.sB = 0;
        gr.C = h->d_T; gr.ldc = n; gr.sC = 0;
        gr.nbatch = 1; gr.alpha0 = 1.0; gr.slices = 1;
        gr.ctl = h->d_ctl; gr.ctl_mode = 2; gr.role = 1;
        {
            TimedLaunch tg(h, s, 2, 2.0 * (double)n * n);   // per unit of rank
            HIPCHK(launch_dgemm(gr, s));
        }
        HIPCHK(launch_lowrank_check(h->d_Dt, h->d_T, n, h->d_pw, h->d_ctl, s));
        // a copy of the decision for the next build's column count and for the counters
        HIPCHK(hipMemcpyAsync(h->h_ctl, h->d_ctl, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
        if (!h->capturing) HIPCHK(hipEventRecord(h->ev_ctl, s));
        return 0;
    };

    // the factor alone on the device (its column steps are single-workgroup
    // launches that any concurrent kernel would hold back), then the
    // reciprocal part and the self term on the side streams
    hipStream_t ls = h->side;
    if (lowrank && h->factor_first) {
        const int frc = run_factor(st);
        if (frc) return frc;
    }
    HIPCHK(hipEventRecord(h->ev_fork, st));
    if (lr_on) HIPCHK(hipStreamWaitEvent(h->side2, h->ev_fork, 0));
    HIPCHK(hipStreamWaitEvent(ls, h->ev_fork, 0));

    // B3/B4: short-range J and K.  Per class pair: the density-weighted
    // screen compacts the neighbour list into FP64 and FP32 work lists, then
    // one launch per list.
    h->st.sr_fold_mask = h->st.sr_kernel_mask = h->st.sr_jengine_mask = 0;
    // without K the J-engine runs: Hermite densities of every pair first (B2)
    const bool jonly = !wantK;
    if ((h->parts & PBC_JK_PART_SR) && jonly) {
        for (int c = 0; c < kNumClass; ++c) {
            HdensArgs ha{};
            ha.pairs = h->d_pairs; ha.groups = h->d_groups;
            ha.g0 = S.class_start[c]; ha.ngroups = S.class_start[c + 1] - S.class_start[c];
            ha.p0 = h->class_p0[c]; ha.Dt = h->d_Dt; ha.nbfc = n; ha.hd = h->d_hd + h->hd_base[c];
            HIPCHK(launch_hdens(c, ha, st));
        }
    }
    if (h->parts & PBC_JK_PART_SR) {
        HIPCHK(launch_fill((double *)h->d_wcnt, 42, 0.0, st));
        SRArgs a{};
        a.pairs = h->d_pairs; a.groups = h->d_groups;
        a.Dt = h->d_Dt; a.Dmax = h->d_Dmax;
        a.X = h->d_X; a.Y = h->d_Y; a.nbfc = n; a.nshell = S.nshell;
        a.lat = lat_args(S);
        a.w2 = S.omega * S.omega; a.d_schwarz = S.d_schwarz; a.d_ewald_R = S.d_ewald_R;
        a.rcap2 = S.r_cut > 0 ? S.r_cut * S.r_cut : 0.0;
        a.fp32_below = S.fp32_below;
        a.boys = h->d_boys; a.bexp = h->d_bexp; a.counters = h->d_cnt;
        a.want_k = wantK ? 1 : 0;
        int slot = 0;
        for (int cb = 0; cb < kNumClass; ++cb)
            for (int ck = cb; ck < kNumClass; ++ck, ++slot) {
                const long e0 = h->nbr_off[slot], e1 = h->nbr_off[slot + 1];
                if (e1 == e0 || !((h->sr_classes >> slot) & 1)) continue;
                // d class pairs whose block does not fit in one lane's registers run
                // the per-lane kernel one component slice at a time, or (tiny cells,
                // and (dd|dd)) one wavefront per group pair (FP64)
                const bool coop = !sr_per_lane(cb, ck);
                const bool sliced = coop && !h->coop_d[slot] && sr_sliceable(cb, ck);
                // mixed precision: the density screen splits the list into FP64
                // and FP32 work lists; otherwise the kernels screen in place.
                // Below kFp32MinL the FP32 kernels save nothing: their quartets'
                // cost is the FP64 screening, sphere and lattice search, and the
                // second launch costs more than the FP32 arithmetic saves.
                const bool split = S.fp32_below > 0 && (!coop || sliced) &&
                                   kClassL[cb] + kClassL[ck] >= h->fp32_min_l;
                PartArgs pa{};
                pa.lat = a.lat;
                pa.groups = h->d_groups; pa.gb0 = S.class_start[cb]; pa.gk0 = S.class_start[ck];
                pa.bra = h->d_nbr_bra + e0; pa.ket = h->d_nbr_ket + e0; pa.n = e1 - e0;
                pa.Dmax = h->d_Dmax; pa.nshell = S.nshell;
                pa.d_schwarz = S.d_schwarz; pa.fp32_below = S.fp32_below;
                pa.split = 1;
                pa.b64 = h->d_w64b + e0; pa.k64 = h->d_w64k + e0;
                pa.b32 = h->d_w32b + e0; pa.k32 = h->d_w32k + e0;
                pa.counts = h->d_wcnt + 2 * slot;
                pa.chunk_counts = h->d_pcc;
                if (split) HIPCHK(launch_partition(pa, st));
                a.slot = slot;
                a.gb0 = S.class_start[cb];
                a.gk0 = S.class_start[ck];
                a.tri = (cb == ck);
                a.max_entries = e1 - e0;
                a.max_prim_pairs = std::max(h->class_max_pp[cb], h->class_max_pp[ck]);
                a.hd_b = h->d_hd + h->hd_base[cb]; a.hd_p0b = h->class_p0[cb];
                a.hd_k = h->d_hd + h->hd_base[ck]; a.hd_p0k = h->class_p0[ck];
                for (int prec = 0; prec < (split ? 2 : 1); ++prec) {
                    a.nbr_bra = !split ? pa.bra : prec ? pa.b32 : pa.b64;
                    a.nbr_ket = !split ? pa.ket : prec ? pa.k32 : pa.k64;
                    a.count = !split ? h->d_ncnt + slot : h->d_wcnt + 2 * slot + prec;
                    // both lists follow the class pair's fold choice: folded, the shifts'
                    // Hermite integrals are summed in FP64 before the transforms; unfolded,
                    // each shift is transformed in the list's precision and added in FP64
                    TimedLaunch tl(h, st, 5 + slot, 0.0);
                    if (h->fold[slot]) h->st.sr_fold_mask |= 1 << slot;
                    if (coop && (h->coop_d[slot] || !sr_sliceable(cb, ck))) h->st.sr_kernel_mask |= 1 << slot;
                    hipError_t e = hipErrorNotSupported;
                    if (jonly && sr_jengine(cb, ck)) {
                        e = launch_sr_j(cb, ck, a, st);
                        if (e == hipSuccess) {
                            h->st.sr_jengine_mask |= 1 << slot;
                            continue;
                        }
                        if (e != hipErrorNotSupported) HIPCHK(e);
                    }
                    if (!coop) e = launch_sr_jk(cb, ck, a, prec == 1, h->fold[slot], st);
                    else if (sliced) e = launch_sr_slices(cb, ck, a, prec == 1, h->fold[slot], st);
                    else e = hipErrorNotSupported;
                    if (e == hipErrorNotSupported && coop) e = launch_sr_coop(cb, ck, a, st);
                    if (e == hipErrorNotSupported) return fail(PBC_JK_ENOTSUP, "d-shell kernels not built");
                    HIPCHK(e);
                }
            }
    }
    if (!h->capturing) HIPCHK(hipEventRecord(h->ev[1], st));
    if (h->serial_lr) {
        // the reciprocal part after the short range instead of beside it
        HIPCHK(hipEventRecord(h->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(ls, h->ev_fork, 0));
    }

    // B6 prelude (side stream, beside the short range): the density factor of
    // the low-rank exchange, whose rank stays on the device.
    if (!h->capturing) HIPCHK(hipEventRecord(h->ev[4], ls));
    SfacArgs sa{};
    sa.pairs = h->d_pairs; sa.sp_start = h->d_sp_start; sa.sp_pairs = h->d_sp_pairs;
    sa.sp_shA = h->d_sp_shA; sa.sp_shB = h->d_sp_shB; sa.sh_l = h->d_sh_l; sa.sh_aoc = h->d_sh_aoc;
    sa.F = h->d_F; sa.nbfc = n; sa.Gs = nullptr;
    // structure factors of one chunk of reciprocal vectors into F, then their
    // J contribution
    auto sfac_j = [&](int g0, int gc, hipStream_t s) -> int {
        if (h->d_F != h->f_clean) {
            HIPCHK(launch_fill(h->d_F, 2L * gc * n2, 0.0, s));
            // the first chunk is the largest: later chunks stay inside the cleared part
            if (g0 == 0 && h->d_F == h->f_own) h->f_clean = h->d_F;
        }
        sa.G = h->d_G + 3 * g0; sa.Gs = h->d_Gs + g0; sa.ng = gc;
        {
            TimedLaunch tl(h, s, 1, 0.0);
            for (int c = 0; c < kNumClass; ++c) {
                sa.sp0 = S.sp_class_start[c];
                sa.nsp = S.sp_class_start[c + 1] - S.sp_class_start[c];
                HIPCHK(launch_sfac(c, sa, s));
            }
        }
        if (wantJ) {
            HIPCHK(launch_dot_batched(h->d_F, h->d_Dt, (int)n2, 2 * gc, h->d_rho, s));
            HIPCHK(launch_jlr(h->d_F, h->d_rho, nullptr, gc, (int)n2, h->d_Jt, s));
        }
        return 0;
    };
    if (lr_on) {
        const int frc = sfac_j(0, std::min(h->gchunk, nG), h->side2);
        if (frc) return frc;
        HIPCHK(hipEventRecord(h->ev_sf, h->side2));
    }
    if (lowrank && !h->factor_first) {
        const int frc = run_factor(ls);
        if (frc) return frc;
    }
    h->lr_cap = cap;
    // The 512-row panels of k_ygemm read each F_G once but hold a whole CU
    // (148 KB of LDS); beside the short-range kernels the 64 x 64 tiles of
    // k_dgemm<2> share the CUs better, so the panels run when the reciprocal
    // part has the device to itself.
    const bool ytall = h->y_tall && (h->y_always || h->serial_lr || !(h->parts & PBC_JK_PART_SR));

    // B5/B6: reciprocal-space J and K (side stream).  Both exchange forms
    // write the upper 64 x 64 tiles of K; with the low-rank form queued the
    // dense products are gated on its failure (and the other way round).
    if (lr_on) {
        const int ntile = (n + kGemmTile - 1) / kGemmTile, upper_tiles = ntile * (ntile + 1) / 2;
        for (int g0 = 0; g0 < nG; g0 += h->gchunk) {
            const int gc = std::min(h->gchunk, nG - g0);
            if (g0 == 0) {
                HIPCHK(hipStreamWaitEvent(ls, h->ev_sf, 0));   // chunk 0 ran on side2
            } else {
                const int frc = sfac_j(g0, gc, ls);
                if (frc) return frc;
            }
            if (!wantK) continue;
            const double nd = (double)n;
            const int nb = 2 * gc;
            if (lowrank) {
                // F_b carries sqrt(W_b), so K += sum_b Y_b Y_b^T with Y_b = F_b L.
                // Y_b^T = L^T F_b (rows j < rank), stored as Y_b by columns:
                // column j of Y_b at T + b n cap + j n.
                GemmArgs g1{};
                g1.M = cap; g1.N = n; g1.K = n;
                g1.A = h->d_L; g1.lda = n; g1.sA = 0;
                g1.B = h->d_F; g1.ldb = n; g1.sB = n2;
                g1.C = h->d_T; g1.ldc = n; g1.sC = (long)n * cap;
                g1.nbatch = nb; g1.alpha0 = 1.0; g1.reduce = 0; g1.slices = 1;
                g1.ctl = h->d_ctl; g1.ctl_mode = 4; g1.role = 2; g1.tile = h->y_tile;
                {
                    TimedLaunch tl(h, ls, 30, 2.0 * nd * nd * nb);   // per unit of rank
                    HIPCHK(ytall ? launch_ygemm(g1, ls) : launch_dgemm(g1, ls));
                    h->st.y_kernel = ytall ? 1 : 0;
                }
                // K += sum_b Y_b Y_b^T on the upper tiles, the batch split into
                // slices (each slice's tile sums added atomically)
                GemmArgs g2{};
                g2.M = g2.N = n; g2.K = cap;
                g2.A = h->d_T; g2.lda = n; g2.sA = (long)n * cap; g2.transA = 1;
                g2.B = h->d_T; g2.ldb = n; g2.sB = (long)n * cap;
                g2.C = h->d_Kt; g2.ldc = n; g2.sC = 0;
                g2.nbatch = nb; g2.alpha0 = 1.0; g2.reduce = 1; g2.upper = 1;
                g2.slices = (int)std::max(1L, std::min<long>(nb, (kStage2Blocks + upper_tiles - 1) / upper_tiles));
                g2.ctl = h->d_ctl; g2.ctl_mode = 2; g2.role = 3;
                {
                    TimedLaunch tl(h, ls, 31, nd * (nd + 1.0) * nb);   // per unit of rank (upper triangle)
                    HIPCHK(launch_dgemm(g2, ls));
                }
            }
            // dense form: T_b = F_b D, K += T_b F_b on the upper tiles (F_b symmetric)
            GemmArgs g1{};
            g1.M = g1.N = g1.K = n;
            g1.A = h->d_F; g1.lda = n; g1.sA = n2;
            g1.B = h->d_Dt; g1.ldb = n; g1.sB = 0;
            g1.C = h->d_T; g1.ldc = n; g1.sC = n2;
            g1.nbatch = nb; g1.alpha = nullptr; g1.alpha0 = 1.0; g1.reduce = 0; g1.slices = 1;
            g1.ctl = h->d_ctl; g1.ctl_mode = lowrank ? 3 : 0;
            {
                TimedLaunch tl(h, ls, lowrank ? 3 : 0, 2.0 * nd * nd * nd * g1.nbatch);
                HIPCHK(launch_dgemm(g1, ls));
            }
            for (int half = 0; half < 2; ++half) {
                GemmArgs g2{};
                g2.M = g2.N = g2.K = n;
                g2.A = h->d_T + (long)half * gc * n2; g2.lda = n; g2.sA = n2;
                g2.B = h->d_F + (long)half * gc * n2; g2.ldb = n; g2.sB = n2;
                g2.C = h->d_Kt; g2.ldc = n; g2.sC = 0;
                g2.nbatch = gc; g2.alpha = nullptr; g2.alpha0 = 1.0; g2.reduce = 1; g2.upper = 1;
                g2.slices = std::max(1, std::min(gc, 2048 / std::max(1, upper_tiles)));
                g2.ctl = h->d_ctl; g2.ctl_mode = lowrank ? 3 : 0;
                TimedLaunch tl(h, ls, lowrank ? 3 : 0, nd * (nd + 1.0) * nd * g2.nbatch);
                HIPCHK(launch_dgemm(g2, ls));
            }
        }
    }
    
    // B7: self term -(pi/(V w^2)) S_bra S_ket
    if (h->parts & PBC_JK_PART_SELF) {
        const double f = -kPi / (S.lat.V * S.omega * S.omega);
        if (wantJ) {
            HIPCHK(launch_fill(h->d_scal, 1, 0.0, ls));
            HIPCHK(launch_dot(h->d_S, h->d_Dt, n2, h->d_scal, ls));
            HIPCHK(launch_axpy_scaled(h->d_Jt, h->d_S, n2, f, h->d_scal, ls));
        }
        if (wantK) {
            GemmArgs g1{};
            g1.M = g1.N = g1.K = n;
            g1.A = h->d_S; g1.lda = n; g1.sA = 0;
            g1.B = h->d_Dt; g1.ldb = n; g1.sB = 0;
            g1.C = h->d_T; g1.ldc = n; g1.sC = 0;
            g1.nbatch = 1; g1.alpha0 = 1.0; g1.reduce = 0; g1.slices = 1;
            const double nd = (double)n;
            {
                TimedLaunch tg(h, ls, 0, 2.0 * nd * nd * nd);
                HIPCHK(launch_dgemm(g1, ls));
            }
            GemmArgs g2 = g1;
            g2.A = h->d_T; g2.B = h->d_S; g2.C = h->d_Kt; g2.alpha0 = f; g2.reduce = 1; g2.upper = 1;
            {
                TimedLaunch tg(h, ls, 0, nd * (nd + 1.0) * nd);
                HIPCHK(launch_dgemm(g2, ls));
            }
        }
    }
    if (!h->capturing) HIPCHK(hipEventRecord(h->ev[5], ls));
    HIPCHK(hipEventRecord(h->ev_join, ls));
    HIPCHK(hipStreamWaitEvent(st, h->ev_join, 0));
    if (!h->capturing) HIPCHK(hipEventRecord(h->ev[2], st));

    // B8: symmetrise, back-transform, energies
    if (wantJ) {
        FinalArgs fa{h->d_X, h->d_Jt, n, nb, 0, h->d_inv_ci, h->d_inv_cc, Jo};
        HIPCHK(launch_final(fa, st));
    }
    if (wantK) {
        FinalArgs fa{h->d_Y, h->d_Kt, n, nb, kGemmTile, h->d_inv_ci, h->d_inv_cc, Ko};
        HIPCHK(launch_final(fa, st));
    }
    if (E_J || E_K) {
        HIPCHK(launch_fill(h->d_scal + 1, 2, 0.0, st));
        if (E_J) HIPCHK(launch_dot(dD, Jo, m2, h->d_scal + 1, st));
        if (E_K) HIPCHK(launch_dot(dD, Ko, m2, h->d_scal + 2, st));
    }
    if (!h->capturing) HIPCHK(hipEventRecord(h->ev[3], st));
    HIPCHK(hipMemcpyAsync(h->h_cnt, h->d_cnt, kNumCounters * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    if (!h->capturing) HIPCHK(hipEventRecord(h->ev_cnt, st));
    h->timed = !h->capturing;
    if ((E_J || E_K) && !h->capturing) {
        double e[2];
        HIPCHK(hipMemcpyAsync(e, h->d_scal + 1, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (E_J) *E_J = 0.5 * e[0];
        if (E_K) *E_K = -0.25 * e[1];
    }
    return 0;
}

// A build that fails part-way leaves no work of its own in flight on the
// side stream.
int run_build(pbc_jk *h, const double *dD, double *dJ, double *dK, double *E_J, double *E_K, hipStream_t st)
{
    const int rc = run_build_streams(h, dD, dJ, dK, E_J, E_K, st);
    if (rc && h->side) (void)hipStreamSynchronize(h->side);
    if (rc && h->side2) (void)hipStreamSynchronize(h->side2);
    return rc;
}

void drop_graph(pbc_jk *h)
{
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
}

// The device part of a host-memory build through a captured graph: the
// first call captures one build (density in d_D; J, K into d_Jo, d_Ko; the
// energies' dot products into d_scal) on the handle's stream, with the fork
// to and join from its side streams, and later calls replay it.  Host-side
// choices (fold and kernel per class pair, the columns queued for the
// density factor) are those of the capture; everything the data decides
// (the factor's rank, the exchange form) stays on the device.
int run_graph(pbc_jk *h, hipStream_t st)
{
    if (!h->gexec) {
        double dummy = 0.0;
        h->cnt_done = event_done(h->ev_cnt);
        h->ctl_done = event_done(h->ev_ctl);
        h->capturing = true;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) {
            h->capturing = false;
            return fail(PBC_JK_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        }
        const int rc = run_build_streams(h, h->d_D, h->d_Jo, h->d_Ko, &dummy, &dummy, st);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(st, &g);
        h->capturing = false;
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e2 != hipSuccess) return fail(PBC_JK_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
        const hipError_t e3 = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) {
            h->gexec = nullptr;
            return fail(PBC_JK_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
        }
    }
    HIPCHK(hipGraphLaunch(h->gexec, st));
    return 0;
}

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

namespace pbcjk {

int handle_new(const pbc_cell *cell, const pbc_atoms *atoms, const pbc_basis *basis, double omega,
               const pbc_jk_thresholds *thr, pbc_jk **out)
{
    *out = nullptr;
    if (!cell || !atoms || !basis) return fail(PBC_JK_EINVAL, "cell, atoms and basis are required");
    double th[8] = {1e-14, 1e-14, 1e-14, 1e-14, 1e-14, 0.0, 0.0, 0.0};
    if (thr) {
        th[0] = thr->pair_R; th[1] = thr->pair_cs; th[2] = thr->ewald_R; th[3] = thr->ewald_K;
        th[4] = thr->schwarz; th[5] = thr->fp32_below; th[6] = thr->r_cut; th[7] = thr->g_cut;
    }
    pbc_jk *h = new (std::nothrow) pbc_jk();
    if (!h) return fail(PBC_JK_ENOMEM, "host allocation failed");
    std::string err;
    int rc;
    try {
        rc = build_setup(cell->a, atoms->natom, atoms->xyz, atoms->charge, basis->nshell, basis->atom, basis->l, basis->pure,
                         basis->nprim, basis->exps, basis->coefs, omega, th, h->S, err);
    } catch (const std::bad_alloc &) {
        delete h;
        return fail(PBC_JK_ENOMEM, "host allocation failed during setup");
    }
    if (rc) {
        delete h;
        return fail(PBC_JK_EINVAL, err);
    }
#if !PBCJK_WITH_D
    for (int s = 0; s < h->S.nshell; ++s)
        if (h->S.sh_l[s] == 2) {
            delete h;
            return fail(PBC_JK_ENOTSUP, "d shells are not supported by this build");
        }
#endif
    const Setup &S = h->S;
    h->st.nbf = S.nbf; h->st.nbf_cart = S.nbfc; h->st.n_pairs = (long)S.pairs.size();
    h->st.n_groups = (long)S.groups.size(); h->st.n_gvec = (int)S.Gw.size(); h->st.omega = S.omega;
    *out = h;
    return 0;
}

size_t handle_fixed_bytes(pbc_jk *h, double lr_budget_mb)
{
    const double keep = h->lr_budget_mb;
    h->lr_budget_mb = lr_budget_mb;
    h->dry = true;
    h->dry_bytes = 0;
    (void)create_device(h);
    h->dry = false;
    h->lr_budget_mb = keep;
    return h->dry_bytes;
}

int handle_device(pbc_jk *h, Arena *arena, bool profile, double lr_budget_mb)
{
    h->arena = arena;
    h->profile = profile;
    h->lr_budget_mb = lr_budget_mb;
    int rc = create_device(h);
    if (rc) {
        std::string keep = g_err;
        release_device(h);
        g_err = keep;
    }
    return rc;
}

void handle_drop_device(pbc_jk *h)
{
    (void)hipSetDevice(h->device);
    drop_graph(h);
    if (h->own) (void)hipStreamSynchronize(h->own);
    if (h->side) (void)hipStreamSynchronize(h->side);
    if (h->side2) (void)hipStreamSynchronize(h->side2);
    release_device(h);
}

size_t handle_nbr_bytes(const pbc_jk *h) { return h->nbr_bytes_needed; }
size_t handle_dev_bytes(const pbc_jk *h) { return h->dev_bytes; }
int handle_natom(const pbc_jk *h) { return (int)h->S.natom; }

void handle_delete(pbc_jk *h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->own) (void)hipStreamSynchronize(h->own);
    if (h->side) (void)hipStreamSynchronize(h->side);
    if (h->side2) (void)hipStreamSynchronize(h->side2);
    release(h);
    delete h;
}

}  // namespace pbcjk

namespace {

// ---------------------------------------------------------------- allocation-free build
// Work buffers of pbc_jk_build_device_static: one file-scope device array
// per GPU (held until the process ends), carved per call.  Host code never
// uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kScratchDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
char *g_scratch_ptr[kScratchDevices] = {};

int scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= kScratchDevices) return fail(PBC_JK_ENOTSUP, "device index above the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PBC_JK_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

// The per-build work buffers of a handle (the setup data, the neighbour
// lists and their per-build work lists stay with the handle).
struct WorkBufs {
    double *D, *Dt, *Dmax, *X, *Y, *Jt, *Kt, *Jo, *Ko, *F, *T, *rho, *scal, *L, *pw, *hd;
    unsigned long long *dmaxg, *cnt, *wcnt;
    int *pwi, *ctl;
    int gchunk;
};

WorkBufs work_of(const pbc_jk *h)
{
    return WorkBufs{h->d_D, h->d_Dt, h->d_Dmax, h->d_X, h->d_Y, h->d_Jt, h->d_Kt, h->d_Jo, h->d_Ko, h->d_F,
                    h->d_T, h->d_rho, h->d_scal, h->d_L, h->d_pw, h->d_hd, h->d_dmaxg, h->d_cnt, h->d_wcnt,
                    h->d_pwi, h->d_ctl, h->gchunk};
}

void set_work(pbc_jk *h, const WorkBufs &w)
{
    h->d_D = w.D; h->d_Dt = w.Dt; h->d_Dmax = w.Dmax; h->d_X = w.X; h->d_Y = w.Y; h->d_Jt = w.Jt;
    h->d_Kt = w.Kt; h->d_Jo = w.Jo; h->d_Ko = w.Ko; h->d_F = w.F; h->d_T = w.T; h->d_rho = w.rho;
    h->d_scal = w.scal; h->d_L = w.L; h->d_pw = w.pw; h->d_hd = w.hd; h->d_dmaxg = w.dmaxg; h->d_cnt = w.cnt;
    h->d_wcnt = w.wcnt; h->d_pwi = w.pwi; h->d_ctl = w.ctl; h->gchunk = w.gchunk;
}

// Carves the work buffers out of [base, base + cap) with the largest
// reciprocal chunk (at most the handle's own) that fits; ENOMEM if even one
// reciprocal vector per chunk does not fit.
int carve_work(const pbc_jk *h, char *base, size_t cap, WorkBufs &w)
{
    const Setup &S = h->S;
    const size_t n = S.nbfc, n2 = n * n, m2 = (size_t)S.nbf * S.nbf, nblk = (n + 63) / 64;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base + off;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    w.D = nullptr;
    w.Dt = (double *)take(8 * n2);
    w.Dmax = (double *)take(8 * (size_t)S.nshell * S.nshell);
    w.X = (double *)take(8 * n2);
    w.Y = (double *)take(8 * n2);
    w.Jt = (double *)take(8 * n2);
    w.Kt = (double *)take(8 * n2);
    w.Jo = (double *)take(8 * m2);
    w.Ko = (double *)take(8 * m2);
    w.scal = (double *)take(8 * 4);
    w.dmaxg = (unsigned long long *)take(8);
    w.cnt = (unsigned long long *)take(8 * kNumCounters);
    w.wcnt = (unsigned long long *)take(8 * 42);
    w.L = (double *)take(8 * n * (size_t)h->lr_rmax);
    w.pw = (double *)take(8 * (n + 2 * nblk + 4));
    w.pwi = (int *)take(4 * 2 * nblk);
    w.ctl = (int *)take(4 * 4);
    w.hd = (double *)take(8 * (size_t)std::max(1L, h->hd_base[kNumClass]));
    if (off > cap) return fail(PBC_JK_ENOMEM, "the cell's work buffers exceed the static scratch array");
    // F and T hold 2 gc matrices each (T at least one), rho 2 gc values
    const size_t per_g = 2 * 8 * n2 * 2 + 2 * 8 + 3 * 256;
    const size_t left = cap - off;
    long gc = (long)std::min<size_t>((size_t)std::max(h->gchunk, 1), left / per_g);
    if (gc < 1) return fail(PBC_JK_ENOMEM, "the cell's work buffers exceed the static scratch array");
    w.F = (double *)take(8 * 2 * (size_t)gc * n2);
    w.T = (double *)take(8 * std::max<size_t>(2 * (size_t)gc * n2, n2));
    w.rho = (double *)take(8 * 2 * (size_t)gc);
    if (off > cap) return fail(PBC_JK_ENOMEM, "the cell's work buffers exceed the static scratch array");
    w.gchunk = (int)gc;
    return 0;
}

}  // namespace

extern "C" {

const char *pbc_jk_last_error(void) { return g_err.c_str(); }

int pbc_jk_create(const pbc_cell *cell, const pbc_atoms *atoms, const pbc_basis *basis, double omega,
                  const pbc_jk_thresholds *thr, pbc_jk **out)
{
    g_err.clear();
    if (!out) return fail(PBC_JK_EINVAL, "out is NULL");
    *out = nullptr;
    auto t0 = std::chrono::steady_clock::now();
    pbc_jk *h = nullptr;
    int rc = pbcjk::handle_new(cell, atoms, basis, omega, thr, &h);
    if (rc) return rc;
    rc = pbcjk::handle_device(h, nullptr, true, 0.0);
    if (rc) {
        std::string keep = g_err;
        pbcjk::handle_delete(h);
        g_err = keep;
        return rc;
    }
    h->st.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return 0;
}

int pbc_jk_build_device(pbc_jk *h, const double *dD, double *dJ, double *dK, double *E_J, double *E_K,
                        void *stream)
{
    g_err.clear();
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    if (!dD) return fail(PBC_JK_EINVAL, "D is NULL");
    HIPCHK(hipSetDevice(h->device));
    auto t0 = std::chrono::steady_clock::now();
    int rc = run_build(h, dD, dJ, dK, E_J, E_K, (hipStream_t)stream);
    h->st.t_build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int pbc_jk_one_electron(pbc_jk *h, double *S_out, double *T_out, double *V_out, double *E_nuc)
{
    g_err.clear();
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    const Setup &S = h->S;
    const bool wantV = V_out || E_nuc;
    if (wantV && S.charge.empty())
        return fail(PBC_JK_EINVAL, "the nuclear attraction and E_nuc need the atom charges (pbc_atoms.charge)");
    HIPCHK(hipSetDevice(h->device));
    hipStream_t st = h->own;
    const int n = S.nbfc, nb = S.nbf;
    const long n2 = (long)n * n, m2 = (long)nb * nb;
    // halves of S, T and V in X, Y, Jt; the reciprocal part and self term of V in Kt
    HIPCHK(launch_fill(h->d_X, n2, 0.0, st));
    HIPCHK(launch_fill(h->d_Y, n2, 0.0, st));
    HIPCHK(launch_fill(h->d_Jt, n2, 0.0, st));
    HIPCHK(launch_fill(h->d_Kt, n2, 0.0, st));
    HIPCHK(launch_fill(h->d_scal, 4, 0.0, st));
    for (int c = 0; c < kNumClass; ++c) {
        OneEArgs oa{};
        oa.pairs = h->d_pairs; oa.groups = h->d_groups;
        oa.g0 = S.class_start[c]; oa.ngroups = S.class_start[c + 1] - S.class_start[c];
        oa.nbfc = n; oa.xyz = h->d_xyz; oa.q = h->d_q; oa.natom = wantV ? S.natom : 0;
        oa.lat = lat_args(S); oa.w2 = S.omega * S.omega; oa.d_ewald_R = S.d_ewald_R;
        oa.rcap2 = S.r_cut > 0 ? S.r_cut * S.r_cut : 0.0;
        oa.boys = h->d_boys; oa.bexp = h->d_bexp;
        oa.XS = h->d_X; oa.XT = h->d_Y; oa.XV = h->d_Jt;
        HIPCHK(launch_one_e(c, oa, st));
    }
    double e_self = 0.0;
    if (wantV) {
        // reciprocal part: the pair structure factors against rho_n(G)
        const int nG = (int)S.Gw.size();
        SfacArgs sa{};
        sa.pairs = h->d_pairs; sa.sp_start = h->d_sp_start; sa.sp_pairs = h->d_sp_pairs;
        sa.sp_shA = h->d_sp_shA; sa.sp_shB = h->d_sp_shB; sa.sh_l = h->d_sh_l; sa.sh_aoc = h->d_sh_aoc;
        sa.F = h->d_F; sa.nbfc = n;
            for (int g0 = 0; g0 < nG; g0 += h->gchunk) {
            const int gc = std::min(h->gchunk, nG - g0);
            sa.G = h->d_G + 3 * g0; sa.Gs = h->d_Gs + g0; sa.ng = gc;
            HIPCHK(launch_fill(h->d_F, 2L * gc * n2, 0.0, st));
            for (int c = 0; c < kNumClass; ++c) {
                sa.sp0 = S.sp_class_start[c];
                sa.nsp = S.sp_class_start[c + 1] - S.sp_class_start[c];
                HIPCHK(launch_sfac(c, sa, st));
            }
            HIPCHK(launch_rho_nuc(h->d_G + 3 * g0, h->d_Gs + g0, gc, h->d_xyz, h->d_q, S.natom, h->d_rho, st));
            HIPCHK(launch_jlr(h->d_F, h->d_rho, nullptr, gc, (int)n2, h->d_Kt, st));
            // E_nuc: 1/2 sum over the half space of |sqrt(W) rho_n|^2
            HIPCHK(launch_dot(h->d_rho, h->d_rho, 2L * gc, h->d_scal + 1, st));
        }
        // self term -(pi/(V w^2)) sum_C q_C S
        double qsum = 0.0, q2 = 0.0;
        for (double z : S.charge) { qsum -= z; q2 += z * z; }
        const double f = -kPi / (S.lat.V * S.omega * S.omega);
        HIPCHK(launch_fill(h->d_scal, 1, qsum, st));
        HIPCHK(launch_axpy_scaled(h->d_Kt, h->d_S, n2, f, h->d_scal, st));
        // E_nuc real space: radius from erfc(x) < (2/sqrt(pi)) e^{-x^2}/x,
        // (2/sqrt(pi)) e^{-w^2 r^2}/(w r^2) = delta_EwaldR
        const double w = S.omega;
        auto tail = [&](double r) { return 2.0 / std::sqrt(kPi) * std::exp(-w * w * r * r) / (w * r * r); };
        double lo = 1e-3, hi = 1.0;
        while (tail(hi) > S.d_ewald_R) hi *= 2.0;
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (lo + hi);
            (tail(m) > S.d_ewald_R ? lo : hi) = m;
        }
        HIPCHK(launch_enuc_real(h->d_xyz, h->d_q, S.natom, lat_args(S), w, hi * hi, h->d_scal + 2, st));
        // self and neutralising-background terms of the point charges
        e_self = -w / std::sqrt(kPi) * q2 - kPi / (2.0 * S.lat.V * w * w) * qsum * qsum;
    }
    double *outs[3] = {S_out, T_out, V_out};
    const double *halves[3] = {h->d_X, h->d_Y, h->d_Jt};
    for (int k = 0; k < 3; ++k) {
        if (!outs[k]) continue;
        FinalArgs fa{halves[k], k == 2 ? h->d_Kt : nullptr, n, nb, 0, h->d_inv_ci, h->d_inv_cc, h->d_Jo};
        HIPCHK(launch_final(fa, st));
        HIPCHK(hipMemcpyAsync(outs[k], h->d_Jo, m2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (E_nuc) {
        double e[2];
        HIPCHK(hipMemcpyAsync(e, h->d_scal + 1, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *E_nuc = 0.5 * e[0] + e[1] + e_self;
    }
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

int pbc_jk_build_device_static(pbc_jk *h, const double *dD, double *dJ, double *dK, double *E_J, double *E_K,
                               void *stream)
{
    g_err.clear();
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    if (!dD) return fail(PBC_JK_EINVAL, "D is NULL");
    HIPCHK(hipSetDevice(h->device));
    char *base = nullptr;
    int rc = scratch_address(h->device, &base);
    if (rc) return rc;
    WorkBufs mine{};
    if ((rc = carve_work(h, base, kScratchBytes, mine))) return rc;
    // the kernels of this build take the scratch addresses; the handle's own
    // buffers are put back once the launches are queued
    const WorkBufs own = work_of(h);
    set_work(h, mine);
    auto t0 = std::chrono::steady_clock::now();
    rc = run_build(h, dD, dJ, dK, E_J, E_K, (hipStream_t)stream);
    h->st.t_build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    set_work(h, own);   // the counters of this build stay readable in the scratch array
    return rc;
}

int pbc_jk_build(pbc_jk *h, const double *D, double *J, double *K, double *E_J, double *E_K)
{
    g_err.clear();
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    if (!D) return fail(PBC_JK_EINVAL, "D is NULL");
    const int nb = h->S.nbf;
    const size_t m2 = (size_t)nb * nb;
    if (!finite_all(D, m2)) return fail(PBC_JK_EINVAL, "D has a non-finite entry");
    double dmax = 0;
    for (size_t i = 0; i < m2; ++i) dmax = std::max(dmax, std::fabs(D[i]));
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < i; ++j)
            if (std::fabs(D[(size_t)i * nb + j] - D[(size_t)j * nb + i]) > 1e-10 * dmax)
                return fail(PBC_JK_EINVAL, "D is not symmetric");
    HIPCHK(hipSetDevice(h->device));
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = h->own;
    HIPCHK(hipMemcpyAsync(h->d_D, D, m2 * sizeof(double), hipMemcpyHostToDevice, st));
    double ej = 0, ek = 0;
    if (h->use_graph) {
        const int rc = run_graph(h, st);
        if (rc) {
            if (h->side) (void)hipStreamSynchronize(h->side);
            if (h->side2) (void)hipStreamSynchronize(h->side2);
            return rc;
        }
        double e[2];
        HIPCHK(hipMemcpyAsync(e, h->d_scal + 1, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ej = 0.5 * e[0];
        ek = -0.25 * e[1];
    } else {
        const int rc = run_build(h, h->d_D, J ? h->d_Jo : nullptr, K ? h->d_Ko : nullptr, E_J ? &ej : nullptr,
                                 E_K ? &ek : nullptr, st);
        if (rc) return rc;
    }
    if (J) HIPCHK(hipMemcpyAsync(J, h->d_Jo, m2 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (K) HIPCHK(hipMemcpyAsync(K, h->d_Ko, m2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (E_J) *E_J = ej;
    if (E_K) *E_K = ek;
    h->st.t_build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return 0;
}

void pbc_jk_destroy(pbc_jk *h) { pbcjk::handle_delete(h); }

int pbc_jk_nbf(const pbc_jk *h)
{
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    return h->S.nbf;
}

int pbc_jk_set_lr(pbc_jk *h, int mode, double tol)
{
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    drop_graph(h);
    if (mode != PBC_JK_LR_AUTO && mode != PBC_JK_LR_DENSE) return fail(PBC_JK_EINVAL, "unknown reciprocal exchange mode");
    if (!(tol < 1.0)) return fail(PBC_JK_EINVAL, "tolerance must be below 1");
    h->lr_mode = mode;
    if (tol > 0.0) h->lr_tol = tol;
    return 0;
}

int pbc_jk_set_sr_classes(pbc_jk *h, int mask21)
{
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    drop_graph(h);
    if (mask21 < 0 || mask21 >= (1 << 21)) return fail(PBC_JK_EINVAL, "class-pair mask has bits above 2^21");
    h->sr_classes = mask21;
    return 0;
}

int pbc_jk_set_graph(pbc_jk *h, int enable)
{
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    HIPCHK(hipSetDevice(h->device));
    if (!enable) {
        if (h->own) HIPCHK(hipStreamSynchronize(h->own));
        drop_graph(h);
    }
    h->use_graph = enable != 0;
    return 0;
}

int pbc_jk_set_parts(pbc_jk *h, int mask)
{
    if (!h) return fail(PBC_JK_EINVAL, "handle is NULL");
    drop_graph(h);
    if (mask & ~7) return fail(PBC_JK_EINVAL, "unknown part bits");
    h->parts = mask;
    return 0;
}

int pbc_jk_stats(const pbc_jk *hc, pbc_jk_counters *out)
{
    if (!hc || !out) return fail(PBC_JK_EINVAL, "handle or out is NULL");
    pbc_jk *h = const_cast<pbc_jk *>(hc);
    if (h->timed) {
        HIPCHK(hipSetDevice(h->device));
        HIPCHK(hipEventSynchronize(h->ev[3]));
        float a = 0, b = 0, c = 0;
        HIPCHK(hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
        HIPCHK(hipEventElapsedTime(&b, h->ev[4], h->ev[5]));
        HIPCHK(hipEventElapsedTime(&c, h->ev[2], h->ev[3]));
        h->st.t_sr_ms = a; h->st.t_lr_ms = b; h->st.t_other_ms = c;
        unsigned long long cnt[kNumCounters];
        HIPCHK(hipMemcpy(cnt, h->stat_cnt ? h->stat_cnt : h->d_cnt, sizeof cnt, hipMemcpyDeviceToHost));
        h->st.quartets = (double)cnt[0];
        h->st.terms = (double)cnt[1];
        h->st.terms_fp32 = (double)cnt[23];
        for (int k = 0; k < 21; ++k) h->st.terms_class[k] = (double)cnt[2 + k];
        int ctl[4] = {0, 1, 0, 0};
        if (h->lr_ran) std::memcpy(ctl, h->h_ctl, sizeof ctl);
        const bool dense = !h->lr_ran || ctl[1];
        const double rank = dense ? 0.0 : (double)ctl[0];
        h->st.lr_rank = dense ? -1.0 : rank;
        // the GEMM figures describe the kernel that accumulated the exchange:
        // k_dgemm<3> (low rank, K += sum_b Y_b Y_b^T) or k_dgemm<0> (dense form,
        // with the self term); the y figures the low-rank products Y_b^T = L^T F_b
        h->st.gemm_kernel = dense ? 0 : 3;
        h->st.t_gemm_ms = h->st.t_sfac_ms = h->st.gemm_flops = h->st.t_chol_ms = 0.0;
        h->st.t_y_ms = h->st.y_flops = 0.0;
        h->st.n_gemm = h->st.n_y = 0;
        for (int k = 0; k < 21; ++k) h->st.t_sr_class_ms[k] = 0.0;
        for (int i = 0; i < h->ntimed; ++i) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, h->tev[2 * i], h->tev[2 * i + 1]));
            const int kind = h->tkind[i];
            const bool main = dense ? (kind == 0 || kind == 3) : kind == 31;
            if (main) {
                h->st.t_gemm_ms += ms;
                h->st.gemm_flops += h->tflops[i] * (kind == 31 ? rank : 1.0);
                h->st.n_gemm++;
            } else if (kind == 30 && !dense) {
                h->st.t_y_ms += ms;
                h->st.y_flops += h->tflops[i] * rank;
                h->st.n_y++;
            } else if (kind == 1) {
                h->st.t_sfac_ms += ms;
            } else if (kind == 4 || kind == 2) {
                h->st.t_chol_ms += ms;   // factorisation and its residual check
            } else if (kind >= 5 && kind < 26) {
                h->st.t_sr_class_ms[kind - 5] += ms;
            }
        }
    }
    *out = h->st;
    return 0;
}

}  // extern "C"
