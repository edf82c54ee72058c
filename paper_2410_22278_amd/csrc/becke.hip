// Periodic Becke partition weights of atom-centred integration-grid points
// (Sec. 2.8, eqs. becke_weight_definition, becke_vicinity_definition,
// becke_mu_definition, becke_switch_definition).
//
// For a point r whose origin atom is A, the atom images taken are those
// within rcut of A's home position (A first); the weight is
//   w(r) = P(A, r) / sum_X P(X, r),  P(X, r) = prod_{Y != X} s(X, Y, r),
//   s = (1 - f(f(f(u)))) / 2,  f(x) = x (3 - x^2) / 2,
//   u = (|r - X| - |r - Y|) / |X - Y|,
// over the images X, Y of that set (the denominator read as a sum over the
// atom images).  P(X, r) is zero once one factor is below delta; the weight is
// zero when P(A, r) is below delta.
//
// One lane per point.  The image list of an atom is built once, on the host,
// at create time.  Points are expected grouped by origin atom: a wavefront
// whose points share one origin reads the image records through the
// constant address space (scalar loads) and walks them in step.  Each lane
// forms the vicinity products of kBeckeBlock images in one pass over the
// partners, so the distance |r - Y| is computed once per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "device_math.h"
#include "kernels.h"
#include "pbcjk.h"

struct pbc_becke {
    int device = 0;
    int natom = 0;
    int max_images = 0;
    long total_images = 0;
    double delta = 0.0;
    double *d_img = nullptr;   // total_images records of 4 doubles (x, y, z, 0)
    int *d_off = nullptr;      // natom + 1 offsets into d_img (in records)
    unsigned long long *d_evals = nullptr;   // switching factors evaluated by the last call
    void *last_stream = nullptr;
};

namespace pbcjk {

namespace {

constexpr int kBeckeBlock = 8;

typedef const __attribute__((address_space(4))) double *CDblPtr;

__device__ __forceinline__ double becke_switch(double u)
{
    const double f1 = 0.5 * u * (3.0 - u * u);
    const double f2 = 0.5 * f1 * (3.0 - f1 * f1);
    const double f3 = 0.5 * f2 * (3.0 - f2 * f2);
    return 0.5 * (1.0 - f3);
}

template <class IP>
__device__ __forceinline__ double becke_point(IP img, int M, const double r[3], double delta, unsigned &evals)
{
    constexpr int NB = kBeckeBlock;
    double num = 0.0, den = 0.0;
    for (int x0 = 0; x0 < M; x0 += NB) {
        double X[NB][3], dX[NB], prod[NB];
        bool live[NB];
        bool any = false;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int x = x0 + j;
            live[j] = x < M;
            prod[j] = 1.0;
            dX[j] = 0.0;
            X[j][0] = X[j][1] = X[j][2] = 0.0;
            if (live[j]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) X[j][c] = img[4 * x + c];
                const double a = r[0] - X[j][0], b = r[1] - X[j][1], e = r[2] - X[j][2];
                dX[j] = sqrt(a * a + b * b + e * e);
                any = true;
            }
        }
        for (int y = 0; y < M && any; ++y) {
            const double Y0 = img[4 * y], Y1 = img[4 * y + 1], Y2 = img[4 * y + 2];
            const double a = r[0] - Y0, b = r[1] - Y1, e = r[2] - Y2;
            const double dY = sqrt(a * a + b * b + e * e);
            any = false;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if (live[j] && x0 + j != y) {
                    ++evals;
                    const double p = X[j][0] - Y0, q = X[j][1] - Y1, t = X[j][2] - Y2;
                    const double u = (dX[j] - dY) * fast_rsqrt(p * p + q * q + t * t);
                    const double s = becke_switch(u);
                    if (s < delta) live[j] = false;
                    else prod[j] *= s;
                }
                any |= live[j];
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int x = x0 + j;
            if (x < M) {
                const double P = live[j] ? prod[j] : 0.0;
                if (x == 0) num = P;
                den += P;
            }
        }
        if (x0 == 0 && num < delta) return 0.0;
    }
    return den > 0.0 ? num / den : 0.0;
}

struct BeckeArgs {
    const double *img;
    const int *off;
    int natom;
    const double *pts;
    const int *origin;
    long npts;
    double delta;
    double *w;
    unsigned long long *evals;   // + switching factors evaluated (summed per wavefront)
};

__global__ __launch_bounds__(256) void k_becke(BeckeArgs a)
{
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool have = g < a.npts;
    int A = have ? a.origin[g] : -1;
    const bool bad = have && (A < 0 || A >= a.natom);
    if (bad) A = -1;
    const int A0 = __builtin_amdgcn_readfirstlane(A);
    const bool uni = __builtin_amdgcn_ballot_w64(have && A != A0) == 0;
    unsigned evals = 0;
    if (have) {
        if (A < 0) {
            a.w[g] = __builtin_nan("");   // origin index out of range
        } else {
            const double r[3] = {a.pts[3 * g], a.pts[3 * g + 1], a.pts[3 * g + 2]};
            const int i0 = a.off[A], M = a.off[A + 1] - i0;
            double w;
            if (uni) {
                const CDblPtr cp = (CDblPtr)a.img + 4L * __builtin_amdgcn_readfirstlane(i0);
                w = becke_point(cp, __builtin_amdgcn_readfirstlane(M), r, a.delta, evals);
            } else {
                w = becke_point(a.img + 4L * i0, M, r, a.delta, evals);
            }
            a.w[g] = w;
        }
    }
    // every lane of the wavefront is active again here
    unsigned long long e = evals;
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if ((threadIdx.x & 63) == 0 && e) atomicAdd(a.evals, e);
}

int becke_fail(int code, const char *msg) { return set_error(code, msg); }

#define BECKE_HIP(expr)                                                        \
    do {                                                                       \
        const hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) return becke_fail(PBC_JK_EDEVICE, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

}  // namespace pbcjk

using namespace pbcjk;

extern "C" int pbc_becke_create(const pbc_cell *cell, int natom, const double *xyz, double rcut, double delta,
                                pbc_becke **out)
{
    if (!out) return becke_fail(PBC_JK_EINVAL, "pbc_becke_create: out is NULL");
    *out = nullptr;
    if (!cell || !xyz || natom < 1) return becke_fail(PBC_JK_EINVAL, "pbc_becke_create: empty cell or atoms");
    if (!(rcut > 0.0) || !std::isfinite(rcut) || !(delta >= 0.0) || !std::isfinite(delta))
        return becke_fail(PBC_JK_EINVAL, "pbc_becke_create: rcut must be positive and delta non-negative");
    const double *M = cell->a;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(M[i])) return becke_fail(PBC_JK_EINVAL, "pbc_becke_create: non-finite cell");
    for (long i = 0; i < 3L * natom; ++i)
        if (!std::isfinite(xyz[i])) return becke_fail(PBC_JK_EINVAL, "pbc_becke_create: non-finite position");
    // inverse of the row matrix of lattice vectors: f = x Minv
    const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                       M[2] * (M[3] * M[7] - M[4] * M[6]);
    if (!(std::fabs(det) > 0.0)) return becke_fail(PBC_JK_EINVAL, "pbc_becke_create: singular cell");
    double Mi[9];
    Mi[0] = (M[4] * M[8] - M[5] * M[7]) / det;
    Mi[1] = (M[2] * M[7] - M[1] * M[8]) / det;
    Mi[2] = (M[1] * M[5] - M[2] * M[4]) / det;
    Mi[3] = (M[5] * M[6] - M[3] * M[8]) / det;
    Mi[4] = (M[0] * M[8] - M[2] * M[6]) / det;
    Mi[5] = (M[2] * M[3] - M[0] * M[5]) / det;
    Mi[6] = (M[3] * M[7] - M[4] * M[6]) / det;
    Mi[7] = (M[1] * M[6] - M[0] * M[7]) / det;
    Mi[8] = (M[0] * M[4] - M[1] * M[3]) / det;
    // a translate n with |v + n M| <= rcut has |f_i + n_i| <= rcut |column i of Minv|
    double span[3];
    for (int i = 0; i < 3; ++i)
        span[i] = std::sqrt(Mi[i] * Mi[i] + Mi[3 + i] * Mi[3 + i] + Mi[6 + i] * Mi[6 + i]);
    std::vector<double> img;
    std::vector<int> off(natom + 1, 0);
    int maxm = 0;
    try {
        for (int a = 0; a < natom; ++a) {
            const double *A = xyz + 3 * a;
            off[a] = (int)(img.size() / 4);
            img.insert(img.end(), {A[0], A[1], A[2], 0.0});
            for (int b = 0; b < natom; ++b) {
                const double v[3] = {xyz[3 * b] - A[0], xyz[3 * b + 1] - A[1], xyz[3 * b + 2] - A[2]};
                long lo[3], hi[3];
                for (int i = 0; i < 3; ++i) {
                    const double f = v[0] * Mi[i] + v[1] * Mi[3 + i] + v[2] * Mi[6 + i];
                    lo[i] = (long)std::floor(-f - rcut * span[i]);
                    hi[i] = (long)std::ceil(-f + rcut * span[i]);
                }
                for (long n0 = lo[0]; n0 <= hi[0]; ++n0)
                    for (long n1 = lo[1]; n1 <= hi[1]; ++n1)
                        for (long n2 = lo[2]; n2 <= hi[2]; ++n2) {
                            if (b == a && n0 == 0 && n1 == 0 && n2 == 0) continue;
                            double Y[3], d2 = 0.0;
                            for (int i = 0; i < 3; ++i) {
                                Y[i] = xyz[3 * b + i] + n0 * M[i] + n1 * M[3 + i] + n2 * M[6 + i];
                                d2 += (Y[i] - A[i]) * (Y[i] - A[i]);
                            }
                            if (d2 <= rcut * rcut) img.insert(img.end(), {Y[0], Y[1], Y[2], 0.0});
                        }
            }
            maxm = std::max(maxm, (int)(img.size() / 4) - off[a]);
            if (img.size() / 4 > (size_t)0x7fffffff) return becke_fail(PBC_JK_ENOMEM, "pbc_becke_create: too many images");
        }
        off[natom] = (int)(img.size() / 4);
    } catch (const std::bad_alloc &) {
        return becke_fail(PBC_JK_ENOMEM, "pbc_becke_create: host allocation failed");
    }
    pbc_becke *b = new (std::nothrow) pbc_becke;
    if (!b) return becke_fail(PBC_JK_ENOMEM, "pbc_becke_create: host allocation failed");
    b->natom = natom;
    b->max_images = maxm;
    b->total_images = off[natom];
    b->delta = delta;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_img, img.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_off, off.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_evals, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemcpy(b->d_img, img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_evals, 0, sizeof(unsigned long long));
    if (e != hipSuccess) {
        (void)hipFree(b->d_img);
        (void)hipFree(b->d_off);
        (void)hipFree(b->d_evals);
        delete b;
        return becke_fail(e == hipErrorOutOfMemory ? PBC_JK_ENOMEM : PBC_JK_EDEVICE, hipGetErrorString(e));
    }
    *out = b;
    return PBC_JK_OK;
}

extern "C" int pbc_becke_weights(pbc_becke *b, long npts, const double *d_pts, const int *d_origin, double *d_w,
                                 void *stream)
{
    if (!b) return becke_fail(PBC_JK_EINVAL, "pbc_becke_weights: NULL plan");
    if (npts < 0) return becke_fail(PBC_JK_EINVAL, "pbc_becke_weights: negative point count");
    if (npts == 0) return PBC_JK_OK;
    if (!d_pts || !d_origin || !d_w) return becke_fail(PBC_JK_EINVAL, "pbc_becke_weights: NULL array");
    BECKE_HIP(hipSetDevice(b->device));
    BeckeArgs a{b->d_img, b->d_off, b->natom, d_pts, d_origin, npts, b->delta, d_w, b->d_evals};
    const long blocks = (npts + 255) / 256;
    if (blocks > 0x7fffffffL) return becke_fail(PBC_JK_EINVAL, "pbc_becke_weights: too many points");
    // the counter is cleared by a kernel on the same stream (a memset node would
    // not replay reliably inside a captured graph)
    BECKE_HIP(launch_fill((double *)b->d_evals, 1, 0.0, (hipStream_t)stream));
    hipLaunchKernelGGL(k_becke, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    BECKE_HIP(hipGetLastError());
    b->last_stream = stream;
    return PBC_JK_OK;
}

extern "C" int pbc_becke_info(const pbc_becke *b, int *max_images, long *total_images)
{
    if (!b) return becke_fail(PBC_JK_EINVAL, "pbc_becke_info: NULL plan");
    if (max_images) *max_images = b->max_images;
    if (total_images) *total_images = b->total_images;
    return PBC_JK_OK;
}

extern "C" int pbc_becke_evaluations(pbc_becke *b, double *evaluations)
{
    if (!b || !evaluations) return becke_fail(PBC_JK_EINVAL, "pbc_becke_evaluations: NULL argument");
    BECKE_HIP(hipSetDevice(b->device));
    BECKE_HIP(hipStreamSynchronize((hipStream_t)b->last_stream));
    unsigned long long e = 0;
    BECKE_HIP(hipMemcpy(&e, b->d_evals, sizeof e, hipMemcpyDeviceToHost));
    *evaluations = (double)e;
    return PBC_JK_OK;
}

extern "C" void pbc_becke_destroy(pbc_becke *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipFree(b->d_img);
    (void)hipFree(b->d_off);
    (void)hipFree(b->d_evals);
    delete b;
}
