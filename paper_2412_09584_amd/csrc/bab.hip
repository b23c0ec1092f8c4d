// Branch and bound over input boxes on the GPU: the per-iteration steps of the planning
// loop (Algorithms 1-2) around the bound pass -- subdomain pick-out and split (the
// branching heuristics of Section 3.1, Eq. lf_pick), the search's sampling and summary
// (Section 3.3), the best-solution update and the pruner (Section 3).
//
// Large selections (pick-out over the whole candidate set, pruning) use device-wide radix
// sort / flagged selection (hipCUB over rocPRIM): stable, so equal keys keep index
// order.  Per-subdomain work (sorting a subdomain's samples, choosing its split
// dimension) runs one block per subdomain in LDS.
#include <hipcub/hipcub.hpp>

#include <cfloat>
#include <cmath>
#include <mutex>
#include <string>

#include "bound.h"
#include "bound_internal.h"

namespace bp {
bound_status set_error(bound_status s, const std::string &msg);   // api.hip
}

// Scratch of the allocation-free pruner (bound_bab_prune_noalloc): the per-block counts,
// then offsets, of up to 4096 blocks of 1024 subdomains (16 KiB).  Every GPU the library
// runs on holds its own copy until the process ends.  Host code passes the address that
// hipGetSymbolAddress returned for the current device, never the symbol itself (that is
// a host-side stand-in, not a device address).
static __device__ __align__(256) int32_t scratch[4096];

struct bound_bab {
    int max_dom = 0, dim = 0, max_samples = 0;
    float *keys = nullptr, *keys_out = nullptr;
    int32_t *vals = nullptr, *vals_out = nullptr;
    uint8_t *flag = nullptr;
    int32_t *count = nullptr;     // device scratch: selection count
    float *mm = nullptr;          // device scratch: min / max of the scaled keys
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    ~bound_bab() {
        for (void *p : {(void *)keys, (void *)keys_out, (void *)vals, (void *)vals_out,
                        (void *)flag, (void *)count, (void *)mm, tmp})
            if (p) (void)hipFree(p);
    }
};

namespace bp {
namespace {

constexpr int TPB = 256;
constexpr int MAX_SAMPLES = 2048;
inline unsigned blocks(long n) { return (unsigned)((n + TPB - 1) / TPB); }

// comparison key: -0 -> +0, NaN -> +inf
__device__ inline float canon(float x) { return x != x ? INFINITY : x + 0.0f; }

__global__ void k_iota_keys(int n, const float *src, float *keys, int32_t *vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        keys[i] = canon(src[i]);
        vals[i] = i;
    }
}

__global__ void k_fill_u8(int n, uint8_t *p, uint8_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// picked[off + t] = sorted[t], t < cnt; those subdomains are marked taken (flag = 0)
__global__ void k_take(int cnt, const int32_t *sorted, int32_t *picked, int off, uint8_t *flag) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) {
        const int i = sorted[t];
        picked[off + t] = i;
        flag[i] = 0;
    }
}

// min / max of the finite f_lo of the subdomains still available (one block)
__global__ void k_minmax(int n, const float *f_lo, const uint8_t *avail, float *mm) {
    __shared__ float smin[TPB], smax[TPB];
    float lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < n; i += TPB) {
        const float v = f_lo[i];
        if (avail[i] && isfinite(v)) {
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mm[0] = smin[0];
        mm[1] = smax[0];
    }
}

// Sort key of the softmax draw (ascending = pick first): s * fl(1/T) - g, each operation
// rounded in FP32, for available subdomains with finite f_lo; FLT_MAX for non-finite
// f_lo, +inf for taken ones.
__global__ void k_gumbel_keys(int n, const float *f_lo, const float *gum, const uint8_t *avail,
                              const float *mm, float inv_t, float *keys, int32_t *vals) {
#pragma clang fp contract(off)   // s * inv_t and the subtraction rounded separately
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    vals[i] = i;
    const float v = f_lo[i];
    if (!avail[i]) {
        keys[i] = INFINITY;
        return;
    }
    if (!isfinite(v)) {
        keys[i] = FLT_MAX;
        return;
    }
    const float lo = mm[0], hi = mm[1];
    const float s = hi > lo ? (v - lo) / (hi - lo) : 0.f;
    keys[i] = canon(s * inv_t - gum[i]);
}

__global__ void k_samples(long total, int M, int d, const float *lo, const float *hi,
                          const float *U, float *S) {
#pragma clang fp contract(off)   // three separately rounded operations, no fused multiply-add
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const long i = e / ((long)M * d);
    const int j = (int)(e % d);
    const float a = lo[i * d + j], b = hi[i * d + j];
    S[e] = a + (b - a) * U[e];
}

// Bitonic sort, by the whole block, of the (canonical value, index) pairs of v[0 .. M)
// in LDS (P2 = M rounded up to a power of two; the padding sorts last): ascending
// value, equal values by index.
__device__ void block_sort(const float *v, int M, int P2, float *sv, int *si) {
    for (int t = threadIdx.x; t < P2; t += TPB) {
        sv[t] = t < M ? canon(v[t]) : INFINITY;
        si[t] = t;
    }
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < P2; t += TPB) {
                const int o = t ^ stride;
                if (o > t) {
                    const bool up = (t & size) == 0;
                    const float va = sv[t], vb = sv[o];
                    const int ia = si[t], ib = si[o];
                    const bool a_gt_b = va > vb || (va == vb && ia > ib);
                    if (a_gt_b == up) {
                        sv[t] = vb; sv[o] = va;
                        si[t] = ib; si[o] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// One block per subdomain: its M samples sorted by value, then f_hi and the k best
// samples.
__global__ void k_search_summary(int M, int P2, int d, const float *values, const float *S, int k,
                                 float *f_hi, float *top) {
    __shared__ float sv[MAX_SAMPLES];
    __shared__ int si[MAX_SAMPLES];
    const long b = blockIdx.x;
    block_sort(values + b * M, M, P2, sv, si);
    if (threadIdx.x == 0) f_hi[b] = values[b * M + si[0]];
    for (long e = threadIdx.x; e < (long)k * d; e += TPB) {
        const int t = (int)(e / d), j = (int)(e - (long)t * d);
        top[(b * k + t) * d + j] = S[(b * M + si[t]) * d + j];
    }
}

// CEM start of box i: mu = u[i / u_div] if it lies in the box, else the centre;
// sigma = half the width.  One thread per box.
__global__ void k_cem_start(int n, int d, const float *lo, const float *hi, const float *u,
                            int u_div, float *mu, float *sigma) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *p = u ? u + (long)(i / u_div) * d : nullptr;
    bool in = p != nullptr;
    for (int j = 0; j < d && in; ++j) in = p[j] >= lo[(long)i * d + j] && p[j] <= hi[(long)i * d + j];
    for (int j = 0; j < d; ++j) {
        const float a = lo[(long)i * d + j], c = hi[(long)i * d + j];
        mu[(long)i * d + j] = in ? p[j] : (a + c) * 0.5f;
        sigma[(long)i * d + j] = (c - a) * 0.5f;
    }
}

// One CEM round's samples (and their copy into the round's slice of the archive).
__global__ void k_cem_samples(long total, int M, int d, const float *lo, const float *hi,
                              const float *mu, const float *sigma, const float *Z, float *S,
                              float *arch, int ld, int a0) {
#pragma clang fp contract(off)   // the product and the sum rounded separately (plain
                                 // operators: the header's __fmul_rn / __fadd_rn may fuse)
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const long i = e / ((long)M * d);
    const int r = (int)(e - i * M * d), m = r / d, j = r - m * d;
    const long o = i * d + j;
    const float u = mu[o] + sigma[o] * Z[e];
    const float v = fminf(fmaxf(u, lo[o]), hi[o]);
    S[e] = v;
    if (arch) arch[((i * ld) + a0 + m) * d + j] = v;
}

// One block per box: the round's values sorted, then mean and deviation of the n_elite
// best samples per coordinate, summed in elite order.
__global__ void k_cem_refit(int M, int P2, int d, const float *values, const float *S, int E,
                            float jitter, float *mu, float *sigma, float *arch_v, int ld, int a0) {
#pragma clang fp contract(off)
    __shared__ float sv[MAX_SAMPLES];
    __shared__ int si[MAX_SAMPLES];
    const long b = blockIdx.x;
    block_sort(values + b * M, M, P2, sv, si);
    const float rE = (float)E;
    for (int j = threadIdx.x; j < d; j += TPB) {
        float s = 0.f;
        for (int r = 0; r < E; ++r) s += S[(b * M + si[r]) * d + j];
        const float m = s / rE;
        float q = 0.f;
        for (int r = 0; r < E; ++r) {
            const float dv = S[(b * M + si[r]) * d + j] - m;
            q += dv * dv;
        }
        mu[b * d + j] = m;
        sigma[b * d + j] = sqrtf(q / rE) + jitter;
    }
    if (arch_v)
        for (int t = threadIdx.x; t < M; t += TPB) arch_v[b * ld + a0 + t] = values[b * M + t];
}

// One block per subdomain: split dimension and the two children.
__global__ void k_split(int d, const float *lo, const float *hi, const float *top, int k,
                        float *clo, float *chi, int32_t *dim_out) {
    __shared__ float sbest[TPB], wbest[TPB];
    __shared__ int jbest[TPB], jw[TPB];
    const long b = blockIdx.x;
    float bs = -1.f, bw = -1.f;
    int bj = 0x7fffffff, bjw = 0x7fffffff;
    for (int j = threadIdx.x; j < d; j += TPB) {
        const float a = lo[b * d + j], c = hi[b * d + j];
        const float mid = __fmul_rn(__fadd_rn(a, c), 0.5f);
        int nlo = 0;
        for (int t = 0; t < k; ++t) nlo += top[(b * k + t) * d + j] <= mid ? 1 : 0;
        const int diff = nlo - (k - nlo);
        const float width = __fsub_rn(c, a);
        const float score = __fmul_rn(width, (float)(diff < 0 ? -diff : diff));
        if (score > bs) { bs = score; bj = j; }          // j ascending per thread
        if (width > bw) { bw = width; bjw = j; }
    }
    sbest[threadIdx.x] = bs; jbest[threadIdx.x] = bj;
    wbest[threadIdx.x] = bw; jw[threadIdx.x] = bjw;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const int o = threadIdx.x + s;
            if (sbest[o] > sbest[threadIdx.x] ||
                (sbest[o] == sbest[threadIdx.x] && jbest[o] < jbest[threadIdx.x])) {
                sbest[threadIdx.x] = sbest[o];
                jbest[threadIdx.x] = jbest[o];
            }
            if (wbest[o] > wbest[threadIdx.x] ||
                (wbest[o] == wbest[threadIdx.x] && jw[o] < jw[threadIdx.x])) {
                wbest[threadIdx.x] = wbest[o];
                jw[threadIdx.x] = jw[o];
            }
        }
        __syncthreads();
    }
    const int js = sbest[0] > 0.f ? jbest[0] : jw[0];
    for (int j = threadIdx.x; j < d; j += TPB) {
        const float a = lo[b * d + j], c = hi[b * d + j];
        const float mid = __fmul_rn(__fadd_rn(a, c), 0.5f);
        clo[(2 * b) * d + j] = a;
        chi[(2 * b) * d + j] = j == js ? mid : c;
        clo[(2 * b + 1) * d + j] = j == js ? mid : a;
        chi[(2 * b + 1) * d + j] = c;
    }
    if (threadIdx.x == 0 && dim_out) dim_out[b] = js;
}

// one block: argmin of f_hi (ties: lower index); strict improvement updates the best
__global__ void k_update_best(int n, const float *f_hi, const float *top, int k, int d, float *best,
                              float *u_best) {
    __shared__ float sv[TPB];
    __shared__ int si[TPB];
    float v = INFINITY;
    int idx = 0x7fffffff;
    for (int i = threadIdx.x; i < n; i += TPB) {
        const float x = canon(f_hi[i]);
        if (x < v) { v = x; idx = i; }
    }
    sv[threadIdx.x] = v;
    si[threadIdx.x] = idx;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const int o = threadIdx.x + s;
            if (sv[o] < sv[threadIdx.x] || (sv[o] == sv[threadIdx.x] && si[o] < si[threadIdx.x])) {
                sv[threadIdx.x] = sv[o];
                si[threadIdx.x] = si[o];
            }
        }
        __syncthreads();
    }
    const bool better = si[0] < n && sv[0] < canon(*best);
    __syncthreads();
    if (!better) return;
    const int i = si[0];
    for (int j = threadIdx.x; j < d; j += TPB) u_best[j] = top[((long)i * k) * d + j];
    if (threadIdx.x == 0) *best = f_hi[i];
}

__global__ void k_zero_i32(int32_t *p) { *p = 0; }

__global__ void k_prune_flags(int n, const float *f_lo, const float *best, uint8_t *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = canon(f_lo[i]) <= canon(*best) ? 1 : 0;
}

// ---- pruner without allocation: stable compaction through per-block counts.
// Block b of the count and scatter kernels covers subdomains [b * PRUNE_TILE, ...);
// the scan kernel turns the block counts into block offsets and writes the total.
constexpr int PRUNE_TILE = 1024;                  // subdomains per block (4 per thread)
constexpr int PRUNE_MAX_BLOCKS = 4096;
constexpr long PRUNE_MAX_N = (long)PRUNE_TILE * PRUNE_MAX_BLOCKS;
static_assert(PRUNE_MAX_BLOCKS == sizeof(::scratch) / sizeof(int32_t), "scratch holds the block counts");

__device__ inline bool kept(const float *f_lo, int i, float b) { return canon(f_lo[i]) <= b; }

__global__ __launch_bounds__(TPB) void k_prune_count(int n, const float *f_lo, const float *best,
                                                     int32_t *counts) {
    __shared__ int wsum[TPB / 64];
    const float b = canon(*best);
    const int i0 = blockIdx.x * PRUNE_TILE;
    int c = 0;
    for (int t = threadIdx.x; t < PRUNE_TILE; t += TPB) {
        const int i = i0 + t;
        c += (i < n && kept(f_lo, i, b)) ? 1 : 0;
    }
    for (int m = 1; m < 64; m <<= 1) c += __shfl_xor(c, m, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < TPB / 64; ++w) s += wsum[w];
        counts[blockIdx.x] = s;
    }
}

// One block: exclusive scan of nb block counts in place, total to *n_keep.
__global__ __launch_bounds__(TPB) void k_prune_scan(int nb, int32_t *counts, int32_t *n_keep) {
    __shared__ int part[TPB];
    const int per = (nb + TPB - 1) / TPB, a = threadIdx.x * per;
    int s = 0;
    for (int k = 0; k < per && a + k < nb; ++k) s += counts[a + k];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < TPB; ++t) {
            const int v = part[t];
            part[t] = run;
            run += v;
        }
        *n_keep = run;
    }
    __syncthreads();
    int run = part[threadIdx.x];
    for (int k = 0; k < per && a + k < nb; ++k) {
        const int v = counts[a + k];
        counts[a + k] = run;
        run += v;
    }
}

// Block b writes its kept subdomains, in index order, from offset counts[b] on: the
// rank of a kept subdomain inside the block is the number of kept ones before it (wave
// ballots, then the waves' and rounds' totals through LDS).
__global__ __launch_bounds__(TPB) void k_prune_scatter(int n, const float *f_lo, const float *best,
                                                       const int32_t *offsets, int32_t *keep) {
    __shared__ int wcnt[PRUNE_TILE / 64];
    const float b = canon(*best);
    const int i0 = blockIdx.x * PRUNE_TILE, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    bool f[PRUNE_TILE / TPB];
    uint64_t m[PRUNE_TILE / TPB];
#pragma unroll
    for (int r = 0; r < PRUNE_TILE / TPB; ++r) {   // round r covers [r * TPB, (r + 1) * TPB)
        const int i = i0 + r * TPB + threadIdx.x;
        f[r] = i < n && kept(f_lo, i, b);
        m[r] = __ballot(f[r]);
        if (lane == 0) wcnt[r * (TPB / 64) + w] = __popcll(m[r]);
    }
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int base = offsets[blockIdx.x];
#pragma unroll
    for (int r = 0; r < PRUNE_TILE / TPB; ++r) {
        // kept subdomains of the (round, wave) segments before this one
        int before = base;
        for (int s = 0; s < r * (TPB / 64) + w; ++s) before += wcnt[s];
        if (f[r]) keep[before + __popcll(m[r] & below)] = i0 + r * TPB + threadIdx.x;
    }
}

std::mutex g_scratch_mu;
int32_t *g_scratch_ptr[64] = {};   // per device: the address of `scratch` on that GPU

hipError_t sort_pairs(bound_bab *b, int n, hipStream_t st) {
    size_t bytes = b->tmp_bytes;
    return hipcub::DeviceRadixSort::SortPairs(b->tmp, bytes, b->keys, b->keys_out, b->vals,
                                              b->vals_out, n, 0, 32, st);
}

hipError_t select_flagged(bound_bab *b, int n, int32_t *out, int32_t *n_out, hipStream_t st) {
    size_t bytes = b->tmp_bytes;
    hipcub::CountingInputIterator<int32_t> it(0);
    return hipcub::DeviceSelect::Flagged(b->tmp, bytes, it, b->flag, out, n_out, n, st);
}

}  // namespace
}  // namespace bp

using bp::set_error;

#define BCHK(x)                                                                         \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) return set_error(BOUND_E_HIP, std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

extern "C" {

bound_status bound_bab_init(int32_t max_dom, int32_t dim, int32_t max_samples, bound_bab **out) {
    if (!out || max_dom < 1 || dim < 1 || max_samples < 1 || max_samples > bp::MAX_SAMPLES)
        return set_error(BOUND_E_ARG, "bound_bab_init: need max_dom, dim >= 1 and 1 <= max_samples <= 2048");
    *out = nullptr;
    bound_bab *b = new bound_bab();
    b->max_dom = max_dom;
    b->dim = dim;
    b->max_samples = max_samples;
    size_t s1 = 0, s2 = 0;
    hipcub::CountingInputIterator<int32_t> it(0);
    bool ok = hipcub::DeviceRadixSort::SortPairs(nullptr, s1, b->keys, b->keys_out, b->vals,
                                                 b->vals_out, max_dom, 0, 32) == hipSuccess &&
              hipcub::DeviceSelect::Flagged(nullptr, s2, it, b->flag, b->vals, b->count,
                                            max_dom) == hipSuccess;
    b->tmp_bytes = s1 > s2 ? s1 : s2;
    ok = ok && hipMalloc(&b->keys, sizeof(float) * max_dom) == hipSuccess &&
         hipMalloc(&b->keys_out, sizeof(float) * max_dom) == hipSuccess &&
         hipMalloc(&b->vals, sizeof(int32_t) * max_dom) == hipSuccess &&
         hipMalloc(&b->vals_out, sizeof(int32_t) * max_dom) == hipSuccess &&
         hipMalloc(&b->flag, max_dom) == hipSuccess &&
         hipMalloc(&b->count, sizeof(int32_t)) == hipSuccess &&
         hipMalloc(&b->mm, 2 * sizeof(float)) == hipSuccess &&
         hipMalloc(&b->tmp, b->tmp_bytes > 0 ? b->tmp_bytes : 1) == hipSuccess;
    if (!ok) {
        delete b;
        return set_error(BOUND_E_NOMEM, "bound_bab_init: device allocation");
    }
    *out = b;
    return BOUND_OK;
}

void bound_bab_destroy(bound_bab *b) { delete b; }

bound_status bound_bab_pick_out(bound_bab *b, int32_t n_dom, const float *f_lo, const float *f_hi,
                                const float *g, int32_t n_pick, float eta, float temperature,
                                int32_t *picked, int32_t *rest, void *stream) {
    if (!b || n_dom < 0 || n_dom > b->max_dom || n_pick < 0 || !(eta >= 0.f && eta <= 1.f) ||
        !(temperature > 0.f) || !(1.0f / temperature < FLT_MAX) ||
        (n_dom > 0 && (!f_lo || !f_hi || !g || !picked || !rest)))
        return set_error(BOUND_E_ARG, "bound_bab_pick_out: bad arguments");
    if (n_dom == 0) return BOUND_OK;
    hipStream_t st = (hipStream_t)stream;
    const int n = n_pick < n_dom ? n_pick : n_dom;
    const int n1 = (int)std::floor((double)eta * (double)n);
    hipLaunchKernelGGL(bp::k_fill_u8, dim3(bp::blocks(n_dom)), dim3(bp::TPB), 0, st, n_dom, b->flag,
                       (uint8_t)1);
    if (n1 > 0) {
        hipLaunchKernelGGL(bp::k_iota_keys, dim3(bp::blocks(n_dom)), dim3(bp::TPB), 0, st, n_dom, f_hi,
                           b->keys, b->vals);
        BCHK(bp::sort_pairs(b, n_dom, st));
        hipLaunchKernelGGL(bp::k_take, dim3(bp::blocks(n1)), dim3(bp::TPB), 0, st, n1, b->vals_out,
                           picked, 0, b->flag);
    }
    if (n - n1 > 0) {
        hipLaunchKernelGGL(bp::k_minmax, dim3(1), dim3(bp::TPB), 0, st, n_dom, f_lo, b->flag, b->mm);
        hipLaunchKernelGGL(bp::k_gumbel_keys, dim3(bp::blocks(n_dom)), dim3(bp::TPB), 0, st, n_dom,
                           f_lo, g, b->flag, b->mm, 1.0f / temperature, b->keys, b->vals);
        BCHK(bp::sort_pairs(b, n_dom, st));
        hipLaunchKernelGGL(bp::k_take, dim3(bp::blocks(n - n1)), dim3(bp::TPB), 0, st, n - n1,
                           b->vals_out, picked, n1, b->flag);
    }
    if (n_dom - n > 0) BCHK(bp::select_flagged(b, n_dom, rest, b->count, st));
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_samples(bound_bab *b, int32_t n, int32_t M, const float *lo, const float *hi,
                               const float *U, float *samples, void *stream) {
    if (!b || n < 0 || M < 1 || (n > 0 && (!lo || !hi || !U || !samples)))
        return set_error(BOUND_E_ARG, "bound_bab_samples: bad arguments");
    const long total = (long)n * M * b->dim;
    if (total == 0) return BOUND_OK;
    hipLaunchKernelGGL(bp::k_samples, dim3(bp::blocks(total)), dim3(bp::TPB), 0, (hipStream_t)stream,
                       total, M, b->dim, lo, hi, U, samples);
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_search_summary(bound_bab *b, int32_t n, int32_t M, const float *values,
                                      const float *samples, int32_t k, float *f_hi, float *top,
                                      void *stream) {
    if (!b || n < 0 || M < 1 || M > b->max_samples || k < 1 || k > M ||
        (n > 0 && (!values || !samples || !f_hi || !top)))
        return set_error(BOUND_E_ARG, "bound_bab_search_summary: bad arguments");
    if (n == 0) return BOUND_OK;
    int P2 = 1;
    while (P2 < M) P2 <<= 1;
    hipLaunchKernelGGL(bp::k_search_summary, dim3(n), dim3(bp::TPB), 0, (hipStream_t)stream, M, P2,
                       b->dim, values, samples, k, f_hi, top);
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_split(bound_bab *b, int32_t n, const float *lo, const float *hi,
                             const float *top, int32_t k, float *child_lo, float *child_hi,
                             int32_t *split_dim, void *stream) {
    if (!b || n < 0 || k < 1 || (n > 0 && (!lo || !hi || !top || !child_lo || !child_hi)))
        return set_error(BOUND_E_ARG, "bound_bab_split: bad arguments");
    if (n == 0) return BOUND_OK;
    hipLaunchKernelGGL(bp::k_split, dim3(n), dim3(bp::TPB), 0, (hipStream_t)stream, b->dim, lo, hi,
                       top, k, child_lo, child_hi, split_dim);
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_cem_start(bound_bab *b, int32_t n, const float *lo, const float *hi,
                                 const float *u, int32_t u_div, float *mu, float *sigma, void *stream) {
    if (!b || n < 0 || u_div < 1 || (n > 0 && (!lo || !hi || !mu || !sigma)))
        return set_error(BOUND_E_ARG, "bound_bab_cem_start: bad arguments");
    if (n == 0) return BOUND_OK;
    hipLaunchKernelGGL(bp::k_cem_start, dim3(bp::blocks(n)), dim3(bp::TPB), 0, (hipStream_t)stream,
                       n, b->dim, lo, hi, u, u_div, mu, sigma);
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_cem_samples(bound_bab *b, int32_t n, int32_t M, const float *lo, const float *hi,
                                   const float *mu, const float *sigma, const float *Z, float *samples,
                                   float *archive, int32_t ld, int32_t a0, void *stream) {
    if (!b || n < 0 || M < 1 || (archive && (a0 < 0 || (long)a0 + M > ld)) ||
        (n > 0 && (!lo || !hi || !mu || !sigma || !Z || !samples)))
        return set_error(BOUND_E_ARG, "bound_bab_cem_samples: bad arguments");
    const long total = (long)n * M * b->dim;
    if (total == 0) return BOUND_OK;
    hipLaunchKernelGGL(bp::k_cem_samples, dim3(bp::blocks(total)), dim3(bp::TPB), 0, (hipStream_t)stream,
                       total, M, b->dim, lo, hi, mu, sigma, Z, samples, archive, ld, a0);
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_cem_refit(bound_bab *b, int32_t n, int32_t M, const float *values,
                                 const float *samples, int32_t n_elite, float jitter, float *mu,
                                 float *sigma, float *archive_values, int32_t ld, int32_t a0,
                                 void *stream) {
    if (!b || n < 0 || M < 1 || M > b->max_samples || n_elite < 1 || n_elite > M ||
        !(jitter >= 0.f) || (archive_values && (a0 < 0 || (long)a0 + M > ld)) ||
        (n > 0 && (!values || !samples || !mu || !sigma)))
        return set_error(BOUND_E_ARG, "bound_bab_cem_refit: bad arguments");
    if (n == 0) return BOUND_OK;
    int P2 = 1;
    while (P2 < M) P2 <<= 1;
    hipLaunchKernelGGL(bp::k_cem_refit, dim3(n), dim3(bp::TPB), 0, (hipStream_t)stream, M, P2, b->dim,
                       values, samples, n_elite, jitter, mu, sigma, archive_values, ld, a0);
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_update_best(bound_bab *b, int32_t n, const float *f_hi, const float *top,
                                   int32_t k, float *best, float *u_best, void *stream) {
    if (!b || n < 0 || k < 1 || !best || !u_best || (n > 0 && (!f_hi || !top)))
        return set_error(BOUND_E_ARG, "bound_bab_update_best: bad arguments");
    if (n == 0) return BOUND_OK;
    hipLaunchKernelGGL(bp::k_update_best, dim3(1), dim3(bp::TPB), 0, (hipStream_t)stream, n, f_hi,
                       top, k, b->dim, best, u_best);
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_prune_noalloc(int32_t n, const float *f_lo, const float *best, int32_t *keep,
                                     int32_t *n_keep, void *stream) {
    if (n < 0 || (long)n > bp::PRUNE_MAX_N || !best || !n_keep || (n > 0 && (!f_lo || !keep)))
        return set_error(BOUND_E_ARG, "bound_bab_prune_noalloc: bad arguments (need 0 <= n <= " +
                                          std::to_string(bp::PRUNE_MAX_N) + ")");
    int dev = 0;
    BCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(BOUND_E_ARG, "bound_bab_prune_noalloc: device id");
    int32_t *scr;
    {
        std::lock_guard<std::mutex> lk(bp::g_scratch_mu);
        if (!bp::g_scratch_ptr[dev]) {
            void *p = nullptr;
            BCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            bp::g_scratch_ptr[dev] = (int32_t *)p;
        }
        scr = bp::g_scratch_ptr[dev];
    }
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(bp::k_zero_i32, dim3(1), dim3(1), 0, st, n_keep);
        BCHK(hipGetLastError());
        return BOUND_OK;
    }
    const int nb = (int)((n + bp::PRUNE_TILE - 1) / bp::PRUNE_TILE);
    hipLaunchKernelGGL(bp::k_prune_count, dim3(nb), dim3(bp::TPB), 0, st, n, f_lo, best, scr);
    hipLaunchKernelGGL(bp::k_prune_scan, dim3(1), dim3(bp::TPB), 0, st, nb, scr, n_keep);
    hipLaunchKernelGGL(bp::k_prune_scatter, dim3(nb), dim3(bp::TPB), 0, st, n, f_lo, best, scr, keep);
    BCHK(hipGetLastError());
    return BOUND_OK;
}

bound_status bound_bab_prune(bound_bab *b, int32_t n, const float *f_lo, const float *best,
                             int32_t *keep, int32_t *n_keep, void *stream) {
    if (!b || n < 0 || n > b->max_dom || !best || !n_keep || (n > 0 && (!f_lo || !keep)))
        return set_error(BOUND_E_ARG, "bound_bab_prune: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(bp::k_zero_i32, dim3(1), dim3(1), 0, st, n_keep);
        BCHK(hipGetLastError());
        return BOUND_OK;
    }
    hipLaunchKernelGGL(bp::k_prune_flags, dim3(bp::blocks(n)), dim3(bp::TPB), 0, st, n, f_lo, best,
                       b->flag);
    BCHK(bp::select_flagged(b, n, keep, n_keep, st));
    BCHK(hipGetLastError());
    return BOUND_OK;
}

}  // extern "C"
