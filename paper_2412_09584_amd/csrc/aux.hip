// Element-wise and small kernels around the MFMA products: relaxation tables (Lemma 1),
// split clamping, box centre / radius, start of a backward pass, split-multiplier
// injection and gradient, final assembly of the bound, the adjoint's start, the
// standalone box concretisation (Theorem 2), Adam, and weight packing.
#include "bound_internal.h"

namespace bp {
namespace {

constexpr int TPB = 256;

inline unsigned blocks_for(long n, int per = TPB) { return (unsigned)((n + per - 1) / per); }

__device__ inline float wave_sum(float x) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// Block-wide sum of two values (256 threads); result valid in thread 0.
__device__ inline void block_sum2(float &a, float &b) {
    __shared__ float sa[4], sb[4];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) { sa[w] = a; sb[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = sa[0] + sa[1] + sa[2] + sa[3];
        b = sb[0] + sb[1] + sb[2] + sb[3];
    }
}

// ReLU layer (0-based, < used) holding global ReLU index jg: the last layer whose offset
// is <= jg (binary search over the layers' offsets).
__device__ inline int layer_of(const LayerShape *ls, int used, long jg) {
    int a = 0, b = used - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (ls[mid].off <= jg) a = mid;
        else b = mid - 1;
    }
    return a;
}

// Row of lo/hi used by an instance; out-of-range indices are clamped so a bad index can
// never read outside the caller's arrays.
__device__ inline long bound_row(const int32_t *bound_of, long inst, int n_bounds) {
    long b = bound_of ? (long)bound_of[inst] : inst;
    return b < 0 ? 0 : (b >= n_bounds ? n_bounds - 1 : b);
}

// internal (y, x, c) index -> C-major index within a layer of C channels, HW pixels
__device__ inline long to_cmajor(long j, int C, int HW) { return (j % C) * HW + j / C; }
__device__ inline long to_internal(long jn, int C, int HW) { return (jn % HW) * C + jn / HW; }

// Lemma 1 for one neuron (boundary reading: active iff l >= 0, else inactive iff u <= 0);
// an unstable neuron's record carries w = k + 1, k its slot in the compact rows of saved
// coefficients (see k_prep_slots).
__device__ inline Relax relax_of(float l, float u, float a, int k) {
    if (l >= 0.f) return make_float4(1.f, 1.f, 0.f, 0.f);
    if (u <= 0.f) return make_float4(0.f, 0.f, 0.f, 0.f);
    const float su = u / (u - l);
    return make_float4(a, su, -l * su, (float)(k + 1));
}

// Slots of the unstable neurons of one ReLU layer under one bound row: the unstable
// neurons in internal order get 0, 1, 2, ... (stable: -1).  The adjoint needs a saved
// coefficient only where the neuron is unstable, so a pass saves G at these slots only.
// Block (row r, layer m); each thread counts a contiguous segment, then the segment
// bases come from a scan of the 256 counts.
__global__ void k_prep_slots(const LayerShape *ls, long n_relu, const float *lo, const float *hi,
                             const int32_t *bound_of, int n_bounds, int per_inst, int32_t *slot,
                             int32_t *inv, int32_t *count) {
    __shared__ int cnt[256];
    const long r = blockIdx.x;
    const LayerShape L = ls[blockIdx.y];
    const long b = per_inst ? bound_row(bound_of, r, n_bounds) : r;
    const float *lr = lo + b * n_relu + L.off, *hr = hi + b * n_relu + L.off;
    const long seg = (L.d + 255) / 256, j0 = threadIdx.x * seg;
    const long j1 = j0 + seg < L.d ? j0 + seg : L.d;
    // unstable flags of n <= 64 neurons from internal index (channel cc, pixel pp) on,
    // which advances; eight neurons' loads are issued at a time
    auto flags = [&](int n, int &cc, long &pp) -> uint64_t {
        uint64_t f = 0;
        for (int u0 = 0; u0 < n; u0 += 8) {
            float a[8], h[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool ok = u0 + u < n;
                const long jn = ok ? (long)cc * L.HW + pp : 0;   // index 0 stands in past the end
                a[u] = lr[jn];
                h[u] = hr[jn];
                if (ok && ++cc == L.C) { cc = 0; ++pp; }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (u0 + u < n && !(a[u] >= 0.f) && !(h[u] <= 0.f)) f |= 1ull << (u0 + u);
        }
        return f;
    };
    const int cs = j0 < L.d ? (int)(j0 % L.C) : 0;
    const long ps = j0 < L.d ? j0 / L.C : 0;
    int c = 0;
    {
        int cc = cs;
        long pp = ps;
        for (long ja = j0; ja < j1; ja += 64)
            c += __popcll(flags(j1 - ja < 64 ? (int)(j1 - ja) : 64, cc, pp));
    }
    cnt[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < 256; ++t) {
            const int v = cnt[t];
            cnt[t] = run;
            run += v;
        }
        count[r * MAX_RELU_LAYERS + blockIdx.y] = run;
    }
    __syncthreads();
    int k = cnt[threadIdx.x];
    int32_t *out = slot + r * n_relu + L.off;
    int32_t *back = inv + r * n_relu + L.off;     // slot -> internal index
    int cc = cs;
    long pp = ps;
    for (long ja = j0; ja < j1; ja += 64) {
        const int n = j1 - ja < 64 ? (int)(j1 - ja) : 64;
        const uint64_t f = flags(n, cc, pp);
        for (int u = 0; u < n; ++u) {
            const bool un = (f >> u) & 1;
            if (un) back[k] = (int32_t)(ja + u);
            out[ja + u] = un ? k++ : -1;
        }
    }
}

// alpha-gradient of ReLU layer L: the adjoint product left each img's contributions
// [G >= 0] G Lambda_bar at the compact slots of its unstable neurons (gc, row stride D);
// one block per instance walks its slots, sums the instance's rows and stores the
// result at the neuron's C-major index.  Slots of split neurons (w = 0) are skipped.
__global__ void k_alpha_grad(int rows, long D, const LayerShape L, int layer, long n_relu,
                             const int32_t *srow, const int32_t *count, const int32_t *inv,
                             const float *gc, float *galpha, long ga_ld, long ga_off) {
    const long inst = blockIdx.x;
    const long r = srow[inst];
    const int cnt = count[r * MAX_RELU_LAYERS + layer];
    const int32_t *iv = inv + r * n_relu + L.off;
    const float *g = gc + inst * rows * D;
    float *ga = galpha + inst * ga_ld + ga_off;
    for (int k = threadIdx.x; k < cnt; k += TPB) {
        const int j = iv[k];
        float acc = 0.f;
        int q = 0;
        // eight rows' loads in flight at once; the sum keeps the row order
        for (; q + 8 <= rows; q += 8) {
            float a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = g[(q + u) * D + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += a[u];
        }
        for (; q < rows; ++q) acc += g[q * D + k];
        // a split neuron's slot holds no contribution of this pass: its entry is
        // overwritten with 0 by k_alpha_split_zero (no per-slot record read here)
        const int c = j % L.C, p = j / L.C;
        ga[(long)c * L.HW + p] = acc;
    }
}

// The alpha-gradient of a split neuron is 0 (its relaxation has no alpha): one thread per
// split entry of the layer.
__global__ void k_alpha_split_zero(int nnz, int layer, const LayerShape L, const int32_t *sp_inst,
                                   const int32_t *sp_layer, const int32_t *sp_j, float *galpha,
                                   long ga_ld, long ga_off) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnz || sp_layer[q] != layer) return;
    const int j = sp_j[q], c = j % L.C, p = j / L.C;
    galpha[(long)sp_inst[q] * ga_ld + ga_off + (long)c * L.HW + p] = 0.f;
}

__global__ void k_count_nonfinite(const float *p, long n, int32_t *cnt) {
    int a = 0, b = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float v = p[i];
        a += v != v;
        b += isinf(v);
    }
    if (a) atomicAdd(cnt, a);
    if (b) atomicAdd(cnt + 1, b);
}

__global__ void k_fill(float *p, long n, float v) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Four values per thread through 16-byte stores (16-byte aligned p, n4 = n / 4).
__global__ void k_fill4(float4 *p, long n4, float v) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) p[i] = make_float4(v, v, v, v);
}

// Relaxation records of one instance: a block covers a tile of one ReLU layer -- P
// pixels x all C channels of a convolutional layer (C <= PREP_TILE), or PREP_TILE
// consecutive neurons of a dense one -- and moves the bounds and alpha, stored C-major,
// into the records, stored pixel-major, through LDS: both the reads and the 16-byte
// record writes are contiguous across the block.  Layers with more channels than a tile
// take one pixel's channels per block with direct (strided) reads.
constexpr int PREP_SH = PREP_TILE + PREP_TILE / 8;  // room for one pad per pixel when C >= 8

__global__ __launch_bounds__(256) void k_prep_tables(const LayerShape *ls, const int32_t *tile0,
                                                     int used, long n_relu,
                                                     const float *lo, const float *hi,
                                                     const int32_t *bound_of, const float *alpha,
                                                     Relax *tab, int32_t *infeas, int n_bounds,
                                                     const int32_t *slot, int per_inst,
                                                     int32_t *srow, int tiles) {
    __shared__ float sh[3 * PREP_SH];
    // consecutive blocks take consecutive tiles of one instance, so the blocks in flight
    // write one contiguous stretch of the record table (and share one bounds row)
    const long inst = blockIdx.x / (unsigned)tiles;
    const int t0 = (int)(blockIdx.x - inst * tiles);
    if (t0 >= tile0[used]) return;
    // the tile's layer: the last m < used with tile0[m] <= t0
    int m = 0, mb = used - 1;
    while (m < mb) {
        const int mid = (m + mb + 1) >> 1;
        if (tile0[mid] <= t0) m = mid;
        else mb = mid - 1;
    }
    const int t = t0 - tile0[m];
    const LayerShape L = ls[m];
    const long b = bound_row(bound_of, inst, n_bounds);
    if (t0 == 0 && threadIdx.x == 0) {
        infeas[inst] = 0;
        srow[inst] = per_inst ? (int32_t)inst : (int32_t)b;
    }
    const float *lr = lo + b * n_relu + L.off, *hr = hi + b * n_relu + L.off;
    const float *ar = alpha ? alpha + inst * n_relu + L.off : nullptr;
    const int32_t *kr = slot + (per_inst ? inst : b) * n_relu + L.off;
    Relax *tr = tab + inst * n_relu + L.off;
    auto record = [&](long j, float l, float u, float a, int32_t k) {
        if (!ar) a = u >= -l ? 1.f : 0.f;
        const Relax r = relax_of(l, u, a, k);
        // streaming store: the table is far larger than the caches and read back later
        typedef float f4 __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store((f4){r.x, r.y, r.z, r.w}, (f4 *)(tr + j));
    };
    if (L.HW == 1) {                        // dense: the two orders coincide
        const long j0 = (long)t * PREP_TILE;
        for (int e = threadIdx.x; e < PREP_TILE; e += 256) {
            const long j = j0 + e;
            if (j < L.d) record(j, lr[j], hr[j], ar ? ar[j] : 0.f, kr[j]);
        }
        return;
    }
    if (L.C > PREP_TILE) {                  // one pixel, a chunk of its channels
        const int nch = (L.C + PREP_TILE - 1) / PREP_TILE;
        const int p = t / nch, c0 = (t - p * nch) * PREP_TILE;
        for (int e = threadIdx.x; e < PREP_TILE && c0 + e < L.C; e += 256) {
            const long jn = (long)(c0 + e) * L.HW + p;
            record((long)p * L.C + c0 + e, lr[jn], hr[jn], ar ? ar[jn] : 0.f, kr[(long)p * L.C + c0 + e]);
        }
        return;
    }
    const int C = L.C, P = PREP_TILE / C, p0 = t * P;
    const int np = L.HW - p0 < P ? L.HW - p0 : P;     // pixels of this tile
    const int CS = C >= 8 ? C + 1 : C;                // LDS pixel stride, odd when padded
    const float rP = 1.0f / (float)P, rC = 1.0f / (float)C;
    constexpr int PER = PREP_TILE / 256;
    // C-major reads: e -> (c, pixel p0 + q), contiguous in q; all of a thread's loads are
    // issued before the first LDS store
    float vl[PER], vh[PER], va[PER];
    int vs[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        // e / P through one FP32 multiply by fl(1 / P): exact for e < 2^21
        const int c = (int)(((float)e + 0.5f) * rP), q = e - c * P;
        vs[k] = -1;
        if (e < C * P && q < np) {
            const long jn = (long)c * L.HW + p0 + q;
            vs[k] = q * CS + c;
            vl[k] = lr[jn];
            vh[k] = hr[jn];
            va[k] = ar ? ar[jn] : 0.f;
        }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k)
        if (vs[k] >= 0) {
            sh[vs[k]] = vl[k];
            sh[PREP_SH + vs[k]] = vh[k];
            sh[2 * PREP_SH + vs[k]] = va[k];
        }
    __syncthreads();
    // pixel-major writes: record p0 * C + e, slot entries loaded first
    int ks[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        ks[k] = e < np * C ? kr[(long)p0 * C + e] : 0;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        if (e < np * C) {
            const int q = (int)(((float)e + 0.5f) * rC), o = e + q * (CS - C);
            record((long)p0 * C + e, sh[o], sh[PREP_SH + o], sh[2 * PREP_SH + o], ks[k]);
        }
    }
}

__global__ void k_prep_splits(const LayerShape *ls, int used, long T, int n_inst, long n_relu,
                              const float *lo, const float *hi, const int32_t *bound_of,
                              const int32_t *off, const int32_t *idx, const int8_t *sign,
                              Relax *tab, int32_t *infeas, int32_t *sp_inst, int32_t *sp_layer,
                              int32_t *sp_j, int32_t *sp_dup, int n_bounds, int stop_m,
                              int stop_relu, float *stop_cen, float *stop_rad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    const long b = bound_row(bound_of, i, n_bounds);
    const int q0 = off[i], q1 = off[i + 1];
    for (int q = q0; q < q1; ++q) {
        const long g = idx[q];
        sp_inst[q] = i;
        sp_layer[q] = -1;
        sp_j[q] = 0;
        sp_dup[q] = 0;
        if (g < 0 || g >= T) continue;  // not a layer this pass relaxes
        const int m = layer_of(ls, used, g);
        const LayerShape L = ls[m];
        const long jn = g - L.off;
        float l = lo[b * n_relu + g], u = hi[b * n_relu + g];
        int first = q;
        for (int q2 = q0; q2 < q1; ++q2) {
            if (idx[q2] != g) continue;
            if (q2 < first) first = q2;
            if (sign[q2] > 0) l = fmaxf(l, 0.f);
            else u = fminf(u, 0.f);
        }
        if (l > u) infeas[i] = 1;
        const long j = to_internal(jn, L.C, L.HW);
        // a split neuron's record carries w = -(q + 1), q its first entry in the
        // instance's list, and that entry's sign in the sign bit of z: the adjoint
        // epilogue writes the entry's beta-gradient -sign * Lambda_bar
        const float wq = -(float)(first + 1);
        const float zs = sign[first] < 0 ? -0.0f : 0.0f;
        tab[(long)i * n_relu + L.off + j] = l >= 0.f ? make_float4(1.f, 1.f, zs, wq)
                                                     : make_float4(0.f, 0.f, zs, wq);
        sp_dup[q] = first != q;   // a repeated entry: k_beta_grad computes it
        if (m == stop_m && stop_cen) {  // the early-stop node's box sees the clamp too
            const float a = stop_relu ? fmaxf(l, 0.f) : l, c = stop_relu ? fmaxf(u, 0.f) : u;
            stop_cen[(long)i * L.d + j] = 0.5f * (a + c);
            stop_rad[(long)i * L.d + j] = 0.5f * (c - a);
        }
        sp_layer[q] = m;
        sp_j[q] = (int32_t)j;
    }
}

// Box of the early-stop node of ReLU layer `L` (internal order): [l, u] of z_s, or
// [ReLU(l), ReLU(u)] of h_s when relu != 0.
__global__ void k_prep_stop_box(long total, LayerShape L, long n_relu, const float *lo,
                                const float *hi, const int32_t *bound_of, int n_bounds, int relu,
                                float *cen, float *rad) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const long inst = e / L.d, j = e - inst * L.d;
    const long b = bound_row(bound_of, inst, n_bounds);
    const long jn = to_cmajor(j, L.C, L.HW);
    float l = lo[b * n_relu + L.off + jn], u = hi[b * n_relu + L.off + jn];
    if (relu) {
        l = fmaxf(l, 0.f);
        u = fmaxf(u, 0.f);
    }
    cen[e] = 0.5f * (l + u);
    rad[e] = 0.5f * (u - l);
}

// I: the index type, 32-bit unsigned whenever the launch has fewer than 2^31 elements
// (cheaper quotients), else long.
template <class I>
__global__ void k_prep_box(long total, long d0, int C0, int HW0, const float *x_lo,
                           const float *x_hi, float *cen, float *rad) {
    const I e = (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x;
    if ((long)e >= total) return;
    const I inst = e / (I)d0, j = e - inst * (I)d0;
    const long jn = (long)(j % (I)C0) * HW0 + (long)(j / (I)C0);
    const float a = x_lo[inst * d0 + jn], b = x_hi[inst * d0 + jn];
    cen[e] = 0.5f * (a + b);
    rad[e] = 0.5f * (b - a);
}

__global__ void k_init_spec(long img0, long n_img, int rows, int rpi, const float *spec, long dk,
                            int Ck, int HWk, float *lam) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_img * dk) return;
    const long li = e / dk, j = e - li * dk;
    const long gimg = img0 + li;
    const long inst = gimg / rpi;
    const int rr = (int)(gimg - inst * rpi);
    const float sg = rr < rows ? 1.f : -1.f;
    const int r = rr < rows ? rr : rr - rows;
    lam[e] = sg * spec[(inst * rows + r) * dk + to_cmajor(j, Ck, HWk)];
}

__global__ void k_init_spec_acc(long img0, long n_img, int rows, int rpi, const float *spec,
                                long dk, int HWk, const float *bias_k, float *s, float *mag,
                                float *low) {
    const long li = blockIdx.x;
    if (li >= n_img) return;
    const long gimg = img0 + li;
    const long inst = gimg / rpi;
    const int rr = (int)(gimg - inst * rpi);
    const float sg = rr < rows ? 1.f : -1.f;
    const int r = rr < rows ? rr : rr - rows;
    const float *row = spec + (inst * rows + r) * dk;
    float a = 0.f, b = 0.f;
    for (long jn = threadIdx.x; jn < dk; jn += blockDim.x) {
        const float t = row[jn] * bias_k[jn / HWk];
        a += t;
        b += fabsf(t);
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        s[li] = sg * a;
        mag[li] = b;
        low[li] = 0.f;
    }
}

template <bool CONC>
__global__ void k_init_identity(const IdentityParams p, long n_img) {
    const long li = blockIdx.x;
    if (li >= n_img) return;
    const long gimg = p.img0 + li;
    const long inst = gimg / p.rpi;
    const long rr = gimg - inst * p.rpi;
    const float sg = rr < p.dk ? 1.f : -1.f;
    const long nr = rr < p.dk ? rr : rr - p.dk;  // C-major neuron of z_k
    int co = 0, oy = 0, ox = 0;
    if (p.kind == 1) {
        const int hw = p.ho * p.wo;
        co = (int)(nr / hw);
        const int q = (int)(nr - (long)co * hw);
        oy = q / p.wo;
        ox = q - oy * p.wo;
    }
    const int hwin = p.hi_ * p.wi;
    float a = 0.f, b = 0.f;
    for (long j = threadIdx.x; j < p.din; j += blockDim.x) {
        const long pix = j / p.ci;
        const int c = (int)(j - pix * p.ci);
        float gval = 0.f;
        if (p.kind == 0) {
            gval = p.W[nr * p.din + (long)c * hwin + pix];
        } else {
            const int iy = (int)(pix / p.wi), ix = (int)(pix - (long)(pix / p.wi) * p.wi);
            const int ky = iy - (oy * p.stride - p.pad), kx = ix - (ox * p.stride - p.pad);
            if (ky >= 0 && ky < p.kh && kx >= 0 && kx < p.kw)
                gval = p.W[(((long)co * p.ci + c) * p.kh + ky) * p.kw + kx];
        }
        gval *= sg;
        if (CONC) {
            const float cc = p.cen[inst * p.din + j], rad = p.rad[inst * p.din + j];
            a += gval * cc - fabsf(gval) * rad;
            b += fabsf(gval) * (fabsf(cc) + rad);
            if (p.emit) p.emit[li * p.din + (long)c * hwin + pix] = gval;
        } else {
            const Relax t = p.tab[inst * p.tab_ld + j];
            float lam = gval >= 0.f ? gval * t.x : gval * t.y;
            // split neuron: the multipliers' term of its first entry (rows = rpi here)
            if (p.bsum && t.w < 0.f) lam -= p.bsum[(long)(-(int)t.w - 1) * p.rpi + rr];
            const float off = gval < 0.f ? gval * t.z : 0.f;
            const float bt = lam * p.bias_m[j % p.chan_m];
            a += bt + off;
            b += fabsf(bt) + fabsf(off);
            p.out[li * p.din + j] = lam;
        }
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        const float bk = sg * p.bias_k[p.kind == 1 ? co : nr];
        if (CONC) {
            p.s[li] = bk;
            p.low[li] = a;
        } else {
            p.s[li] = bk + a;
            p.low[li] = 0.f;
        }
        p.mag[li] = fabsf(bk) + b;
    }
}

__global__ void k_beta_sum(int nnz, int rows, const int32_t *off, const int32_t *idx,
                           const int8_t *sign, const int32_t *sp_inst, const int32_t *sp_layer,
                           const int32_t *sp_dup, const float *beta, float *bsum) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)nnz * rows) return;
    const int q = (int)(e / rows), r = (int)(e - (long)q * rows);
    // entries this pass does not relax, and repeats (their term is in the first entry's)
    if (sp_layer[q] < 0 || sp_dup[q]) return;
    const int i = sp_inst[q], g = idx[q];
    float s = 0.f;
    for (int q2 = off[i]; q2 < off[i + 1]; ++q2)
        if (idx[q2] == g) s += (float)sign[q2] * beta[(long)q2 * rows + r];
    bsum[e] = s;
}

__global__ void k_finalize(long img0, long n_img, int rows, int rpi, const float *s,
                           const float *low, const float *mag, const int32_t *infeas, int slack,
                           float *lower, float *upper, long ld, float *offset, float *offset_mag,
                           float *best, float *best_upper) {
    const long li = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= n_img) return;
    const long gimg = img0 + li;
    const long inst = gimg / rpi;
    const int rr = (int)(gimg - inst * rpi);
    if (offset) offset[gimg] = s[li];
    if (offset_mag) offset_mag[gimg] = mag[li];
    if (!lower) return;
    float v = s[li] + low[li];
    if (slack) v -= KAPPA_U * mag[li];
    if (infeas[inst]) v = INFINITY;
    if (rr < rows) {
        lower[inst * ld + rr] = v;
        if (best) best[inst * ld + rr] = fmaxf(best[inst * ld + rr], v);
    } else if (upper) {
        upper[inst * ld + rr - rows] = -v;
        if (best_upper)
            best_upper[inst * ld + rr - rows] = fminf(best_upper[inst * ld + rr - rows], -v);
    }
}

__global__ void k_adj_init(long n_img, int rows, long d0, const float *gl, const float *g1,
                           const float *cen, const float *rad, const int32_t *infeas,
                           float *gbar, float *sbar) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_img * d0) return;
    const long img = e / d0, j = e - img * d0;
    const long inst = img / rows;
    const float w = infeas[inst] ? 0.f : gl[img];
    if (j == 0) sbar[img] = w;
    const float g = g1[e];
    const float sg = g > 0.f ? 1.f : (g < 0.f ? -1.f : 0.f);
    gbar[e] = w * (cen[inst * d0 + j] - sg * rad[inst * d0 + j]);
}

// The same, four consecutive inputs per thread (d0 % 4 == 0): 16-byte loads and stores.
__global__ void k_adj_init4(long n_img, int rows, long d0, const float *gl, const float *g1,
                            const float *cen, const float *rad, const int32_t *infeas,
                            float *gbar, float *sbar) {
    // 32-bit quotients: the launch keeps n_img * d0 / 4 below 2^31
    const unsigned e4 = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned q = (unsigned)(d0 >> 2);
    if (e4 >= (unsigned)n_img * q) return;
    const long img = e4 / q, j = (long)(e4 - (unsigned)img * q) * 4;
    const long inst = (unsigned)img / (unsigned)rows;
    // every load issued before the first use
    const int bad = infeas[inst];
    const float glv = gl[img];
    const float4 g = *(const float4 *)(g1 + img * d0 + j);
    const float4 c = *(const float4 *)(cen + inst * d0 + j);
    const float4 r = *(const float4 *)(rad + inst * d0 + j);
    const float w = bad ? 0.f : glv;
    if (j == 0) sbar[img] = w;
    auto one = [&](float gv, float cv, float rv) {
        const float sg = gv > 0.f ? 1.f : (gv < 0.f ? -1.f : 0.f);
        return w * (cv - sg * rv);
    };
    *(float4 *)(gbar + img * d0 + j) =
        make_float4(one(g.x, c.x, r.x), one(g.y, c.y, r.y), one(g.z, c.z, r.z), one(g.w, c.w, r.w));
}

__global__ void k_beta_grad(int nnz, int rows, int layer, const BetaGradLayer L,
                            const int32_t *sp_inst, const int32_t *sp_layer, const int32_t *sp_j,
                            const int32_t *sp_dup, const int8_t *sign, const float *gbar_m,
                            const float *sbar, float *gbeta) {
    // one wave per split entry, its rows in turn: most entries leave at once
    const long q = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (q >= nnz) return;
    // first entries of a neuron get their gradient in the adjoint product's epilogue
    if (sp_layer[q] != layer || !sp_dup[q]) return;
    for (int r = 0; r < rows; ++r) {
        const long img = (long)sp_inst[q] * rows + r;
        const float *gb = gbar_m + img * L.din;
        const long j = sp_j[q];
        float acc = 0.f;
        int bidx;
        if (L.kind == 0) {
            const int hwin = L.hi_ * L.wi;
            const float *wrow = L.W + j * L.din;
            for (long k = lane; k < L.din; k += 64) {
                const long pix = k / L.ci;
                const int c = (int)(k - pix * L.ci);
                acc += gb[k] * wrow[(long)c * hwin + pix];
            }
            bidx = (int)j;
        } else {
            const long pix = j / L.co;
            const int co = (int)(j - pix * L.co);
            const int oy = (int)(pix / L.wo), ox = (int)(pix - (long)oy * L.wo);
            const int taps = L.kh * L.kw * L.ci;
            for (int t = lane; t < taps; t += 64) {
                const int ci = t % L.ci, kk = t / L.ci;
                const int ky = kk / L.kw, kx = kk - ky * L.kw;
                const int y = oy * L.stride - L.pad + ky, x = ox * L.stride - L.pad + kx;
                if (y < 0 || y >= L.hi_ || x < 0 || x >= L.wi) continue;
                acc += gb[((long)y * L.wi + x) * L.ci + ci] *
                       L.W[(((long)co * L.ci + ci) * L.kh + ky) * L.kw + kx];
            }
            bidx = co;
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            const float lam_bar = acc + sbar[img] * L.bias[bidx];
            gbeta[q * rows + r] = -(float)sign[q] * lam_bar;
        }
    }
}

// lower/mag[img] += sum_j lam c - |lam| r, sum_j |lam| (|c| + r) over one row of internal-order
// coefficients, c / r the per-instance box (early stop over a pre-activation box).
__global__ void k_box_conc(long img0, int rpi, long D, const float *lam, const float *cen,
                           const float *rad, float *low, float *mag, float *save) {
    const long li = blockIdx.x;
    const long inst = (img0 + li) / rpi;
    const float *row = lam + li * D;
    const float *c = cen + inst * D, *r = rad + inst * D;
    float a = 0.f, b = 0.f;
    for (long j = threadIdx.x; j < D; j += blockDim.x) {
        const float w = row[j];
        a += w * c[j] - fabsf(w) * r[j];
        b += fabsf(w) * (fabsf(c[j]) + r[j]);
        if (save) save[li * D + j] = w;
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        low[li] += a;
        mag[li] += b;
    }
}

// Adjoint at an early stop over the pre-activation box of layer m: lam_bar = s_bar (c -
// sign(lam) r), then the reverse of the relaxation of layer m (G_bar_{m+1}, alpha-grad).
__global__ void k_adj_stop_linear(long n_img, int rows, long D, const float *lam, const float *g,
                                  const float *cen, const float *rad, const float *gl,
                                  const int32_t *infeas, float *sbar, const Relax *tab, long tab_ld,
                                  float *gout, float *gc, int C, int HW) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_img * D) return;
    const long img = e / D, j = e - img * D;
    const long inst = img / rows;
    const float sb = infeas[inst] ? 0.f : gl[img];
    if (j == 0) sbar[img] = sb;
    const float l = lam[e];
    const float sg = l > 0.f ? 1.f : (l < 0.f ? -1.f : 0.f);
    const float v = sb * (cen[inst * D + j] - sg * rad[inst * D + j]);
    const Relax t = tab[inst * tab_ld + j];
    // saved coefficients exist at the unstable neurons only (slot w - 1); elsewhere the
    // record has equal slopes and no intercept, so the sign of G does not matter
    const float gv = t.w > 0.f ? g[img * D + (int)t.w - 1] : 0.f;
    if (gout) gout[e] = v * (gv >= 0.f ? t.x : t.y) + (gv < 0.f ? sb * t.z : 0.f);
    if (t.w > 0.f) gc[img * D + (int)t.w - 1] = gv >= 0.f ? gv * v : 0.f;   // see k_alpha_grad
}

__global__ void k_beta_grad_stop(int nnz, int rows, int layer, long D, const int32_t *sp_inst,
                                 const int32_t *sp_layer, const int32_t *sp_j, const int8_t *sign,
                                 const float *lam, const float *cen, const float *rad,
                                 const float *sbar, float *gbeta) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)nnz * rows) return;
    const int q = (int)(e / rows), r = (int)(e - (long)q * rows);
    if (sp_layer[q] != layer) return;
    const long inst = sp_inst[q];
    const long img = inst * rows + r;
    const long j = sp_j[q];
    const float l = lam[img * D + j];
    const float sg = l > 0.f ? 1.f : (l < 0.f ? -1.f : 0.f);
    const float lam_bar = sbar[img] * (cen[inst * D + j] - sg * rad[inst * D + j]);
    gbeta[(long)q * rows + r] = -(float)sign[q] * lam_bar;
}

// C-major rows -> internal (channels-last) rows.
__global__ void k_to_internal(long total, long D, int C, int HW, const float *x, float *y) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const long img = e / D, j = e - img * D;
    y[e] = x[img * D + to_cmajor(j, C, HW)];
}

// Per subdomain and neuron: min / max of z over its per_sub sample rows (written C-major
// at lo/hi[sub*ld + j], merged with the values there when `merge`); then z <- ReLU(z) in
// place for the next layer, or a copy of the last layer's output to `out` (C-major).
__global__ void k_sample_minmax(long n_sub, int per_sub, long D, int C, int HW, float *z, float *lo,
                                float *hi, long ld, int relu, float *out, int merge) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_sub * D) return;
    const long sub = e / D, j = e - sub * D;
    float mn = INFINITY, mx = -INFINITY;
    for (int s = 0; s < per_sub; ++s) {
        const long o = (sub * per_sub + s) * D + j;
        const float v = z[o];
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
        if (relu) z[o] = fmaxf(v, 0.f);
        if (out) out[(sub * per_sub + s) * D + to_cmajor(j, C, HW)] = v;
    }
    if (lo) {
        const long o = sub * ld + to_cmajor(j, C, HW);
        lo[o] = merge ? fminf(lo[o], mn) : mn;
        hi[o] = merge ? fmaxf(hi[o], mx) : mx;
    }
}

// One projected Adam step of one parameter p with gradient g (moments m, v updated in
// place); shared by the dense step and the fused alpha step, so both round alike.
__device__ inline float adam_elem(float p, float g, float &m, float &v, const AdamArgs &a) {
    const float gr = a.gs * g;
    m = a.b1 * m + (1.f - a.b1) * gr;
    v = a.b2 * v + (1.f - a.b2) * gr * gr;
    const float x = p - (a.lr / a.bc1) * m / (sqrtf(v) / a.bc2s + a.eps);
    return fminf(fmaxf(x, a.lo), a.hi);
}

__global__ void k_adam(long n, float *p, const float *g, float *m, float *v, const AdamArgs a) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float pi = p[i];   // loaded with the others, ahead of the moment stores
    float mi = m[i], vi = v[i];
    const float x = adam_elem(pi, g[i], mi, vi, a);
    m[i] = mi;
    v[i] = vi;
    p[i] = x;
}

// Split neurons keep the slot they have as unstable neurons but take no alpha: their
// slots' row contributions are cleared, so the fused step below sees a zero gradient
// there, as the dense gradient has.  One thread per (split entry, row).
__global__ void k_split_gc_zero(int nnz, int rows, int layer, long D, long n_relu, long off,
                                const int32_t *sp_inst, const int32_t *sp_layer,
                                const int32_t *sp_j, const int32_t *srow, const int32_t *slot,
                                float *gc) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nnz * rows) return;
    const int q = (int)(t / rows), r = (int)(t - (long)q * rows);
    if (sp_layer[q] != layer) return;
    const long inst = sp_inst[q];
    const int s = slot[(long)srow[inst] * n_relu + off + sp_j[q]];
    if (s >= 0) gc[(inst * rows + r) * D + s] = 0.f;
}

// alpha-gradient of ReLU layer L fused with the Adam step on alpha: as k_alpha_grad, the
// block of an instance sums its rows' contributions at each slot (in the same order),
// then steps the neuron's alpha (C-major index) with moments kept at the slot's index.
__global__ void k_alpha_adam(int rows, long D, const LayerShape L, int layer, long n_relu,
                             const int32_t *srow, const int32_t *count, const int32_t *inv,
                             const float *gc, float *alpha, float *m, float *v, long ld, long aoff,
                             const AdamArgs a) {
    const long inst = blockIdx.x;
    const long r = srow[inst];
    const int cnt = count[r * MAX_RELU_LAYERS + layer];
    const int32_t *iv = inv + r * n_relu + L.off;
    const float *g = gc + inst * rows * D;
    float *al = alpha + inst * ld + aoff, *mm = m + inst * ld + aoff, *vv = v + inst * ld + aoff;
    for (int k = threadIdx.x; k < cnt; k += TPB) {
        const int j = iv[k];
        const int c = j % L.C, p = j / L.C;
        const long ai = (long)c * L.HW + p;
        const float pi = al[ai];        // issued ahead of the row loads
        float mi = mm[k], vi = vv[k];
        float acc = 0.f;
        int q = 0;
        for (; q + 8 <= rows; q += 8) {
            float t8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t8[u] = g[(q + u) * D + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += t8[u];
        }
        for (; q < rows; ++q) acc += g[q * D + k];
        const float x = adam_elem(pi, acc, mi, vi, a);
        mm[k] = mi;
        vv[k] = vi;
        al[ai] = x;
    }
}

// One block per (instance, row): reads the row once, coalesced.
// One block per instance: the box (centre, radius) of each of the thread's input
// elements is formed once and serves all the instance's rows, CROWS rows at a time, whose
// coefficient loads are all in flight together; the rows' two sums are then reduced over
// the block.
constexpr int CROWS = 12;
__global__ __launch_bounds__(256) void k_concretize(int rows, long d0, const float *coeff,
                                                   const float *offset, const float *offset_mag,
                                                   const float *x_lo, const float *x_hi, int slack,
                                                   float *lower) {
    __shared__ float red[4][2 * CROWS];
    const long inst = blockIdx.x;
    const float *lo = x_lo + inst * d0, *hi = x_hi + inst * d0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r0 = 0; r0 < rows; r0 += CROWS) {
        const int nr = rows - r0 < CROWS ? rows - r0 : CROWS;
        const float *cr = coeff + (inst * rows + r0) * d0;
        float a[CROWS], b[CROWS];
#pragma unroll
        for (int q = 0; q < CROWS; ++q) a[q] = b[q] = 0.f;
        for (long j = threadIdx.x; j < d0; j += TPB) {
            const float l = lo[j], h = hi[j];
            float w[CROWS];
#pragma unroll
            for (int q = 0; q < CROWS; ++q) w[q] = q < nr ? cr[q * d0 + j] : 0.f;
            const float c = 0.5f * (l + h), r = 0.5f * (h - l), m = fabsf(c) + r;
#pragma unroll
            for (int q = 0; q < CROWS; ++q) {
                a[q] += w[q] * c - fabsf(w[q]) * r;
                b[q] += fabsf(w[q]) * m;
            }
        }
#pragma unroll
        for (int q = 0; q < CROWS; ++q) {
            a[q] = wave_sum(a[q]);
            b[q] = wave_sum(b[q]);
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < CROWS; ++q) {
                red[wave][q] = a[q];
                red[wave][CROWS + q] = b[q];
            }
        }
        __syncthreads();
        if (threadIdx.x < nr) {
            const int q = threadIdx.x;
            const float A = red[0][q] + red[1][q] + red[2][q] + red[3][q];
            const float M = red[0][CROWS + q] + red[1][CROWS + q] + red[2][CROWS + q] + red[3][CROWS + q];
            const long row = inst * rows + r0 + q;
            float v = A + offset[row];
            if (slack) v -= KAPPA_U * (M + (offset_mag ? offset_mag[row] : 0.f));
            lower[row] = v;
        }
        __syncthreads();
    }
}

__global__ void k_pack_T(const float *W, int kind, int ci, int hwin, int co, int kh, int kw,
                         int stride, int ky0, int kx0, int Ty, int Tx, int N, int K, int Kp,
                         long total, float *Bt) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const long n = e / Kp;
    const int k = (int)(e - n * Kp);
    float v = 0.f;
    if (n < N && k < K) {
        if (kind == 0) {  // Bt[n][k] = W[k][cmajor(n)]
            const long pix = n / ci;
            const int c = (int)(n - pix * ci);
            v = W[(long)k * N + (long)c * hwin + pix];
        } else {          // k = (t'y * Tx + t'x) * co + o
            const int o = k % co, tt = k / co;
            const int ty = tt / Tx, tx = tt - ty * Tx;
            const int ky = ky0 + stride * (Ty - 1 - ty), kx = kx0 + stride * (Tx - 1 - tx);
            if (ky < kh && kx < kw) v = W[(((long)o * ci + n) * kh + ky) * kw + kx];
        }
    }
    Bt[e] = v;
}

__global__ void k_pack_F(const float *W, int kind, int ci, int hwin, int kh, int kw, int N, int K,
                         int Kp, long total, float *Bt) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const long n = e / Kp;
    const int k = (int)(e - n * Kp);
    float v = 0.f;
    if (n < N && k < K) {
        if (kind == 0) {  // Bt[n][k] = W[n][cmajor(k)]
            const long pix = k / ci;
            const int c = (int)(k - pix * ci);
            v = W[n * K + (long)c * hwin + pix];
        } else {          // k = (ky * kw + kx) * ci + c
            const int c = k % ci, tt = k / ci;
            const int ky = tt / kw, kx = tt - ky * kw;
            v = W[((n * ci + c) * kh + ky) * kw + kx];
        }
    }
    Bt[e] = v;
}

}  // namespace

hipError_t launch_count_nonfinite(const float *p, long n, int32_t *cnt, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const long nb = blocks_for(n) < 4096 ? blocks_for(n) : 4096;
    hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)nb), dim3(TPB), 0, st, p, n, cnt);
    return hipGetLastError();
}

// One wave per img: lane l sums slots l, l + 64, ... in order, then a fixed xor tree.
__global__ void k_det_reduce(long n_img, long nslot, const float *part, float *s, float *mag) {
    const long img = (long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (img >= n_img) return;
    const float *p = part + img * nslot * 2;
    float a = 0.f, b = 0.f;
    for (long k = lane; k < nslot; k += 64) {
        a += p[2 * k];
        b += p[2 * k + 1];
    }
#pragma unroll
    for (int mk = 32; mk > 0; mk >>= 1) {
        a += __shfl_xor(a, mk, 64);
        b += __shfl_xor(b, mk, 64);
    }
    if (lane == 0) {
        s[img] += a;
        mag[img] += b;
    }
}

hipError_t launch_det_reduce(long n_img, long nslot, const float *part, float *s, float *mag,
                             hipStream_t st) {
    if (n_img <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_det_reduce, dim3((unsigned)((n_img + 3) / 4)), dim3(256), 0, st, n_img,
                       nslot, part, s, mag);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, long n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n % 4 == 0 && ((uintptr_t)p & 15) == 0)
        hipLaunchKernelGGL(k_fill4, dim3(blocks_for(n / 4)), dim3(TPB), 0, st, (float4 *)p, n / 4, v);
    else
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(TPB), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_prep_tables(const NetShapes &ns, int used, int n_inst, long n_relu,
                              const float *lo, const float *hi, const int32_t *bound_of,
                              const float *alpha, Relax *tab, int32_t *infeas, int n_bounds,
                              int32_t *slot, int32_t *slot_inv, int32_t *slot_count,
                              int32_t *srow, int max_rows, hipStream_t st) {
    const long T = used > 0 ? ns.l[used - 1].off + ns.l[used - 1].d : 0;
    if (T == 0) return launch_fill((float *)infeas, n_inst, 0.f, st);  // 0.0f is all-zero bits
    // slots per bound row when the rows fit the slot table, else per instance
    const bool per_inst = bound_of == nullptr || n_bounds > max_rows;
    const int rows = per_inst ? n_inst : n_bounds;
    hipLaunchKernelGGL(k_prep_slots, dim3((unsigned)rows, (unsigned)used), dim3(256), 0, st, ns.dev,
                       n_relu, lo, hi, bound_of, n_bounds, per_inst ? 1 : 0, slot, slot_inv,
                       slot_count);
    long tiles = 0;
    for (int m = 0; m < used; ++m) tiles += prep_tiles(ns.l[m]);
    if (tiles * n_inst > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_prep_tables, dim3((unsigned)(tiles * n_inst)), dim3(256), 0, st, ns.dev,
                       ns.tile0, used, n_relu, lo, hi, bound_of, alpha, tab, infeas, n_bounds, slot,
                       per_inst ? 1 : 0, srow, (int)tiles);
    return hipGetLastError();
}

hipError_t launch_alpha_grad(int n_inst, int rows, long D, const LayerShape &L, int layer,
                             long n_relu, const int32_t *srow, const int32_t *slot_count,
                             const int32_t *slot_inv, const float *gc, float *galpha, long ga_ld,
                             long ga_off, int nnz, const int32_t *sp_inst, const int32_t *sp_layer,
                             const int32_t *sp_j, hipStream_t st) {
    if (n_inst <= 0 || D <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alpha_grad, dim3((unsigned)n_inst), dim3(TPB), 0, st, rows, D, L, layer,
                       n_relu, srow, slot_count, slot_inv, gc, galpha, ga_ld, ga_off);
    if (nnz > 0)
        hipLaunchKernelGGL(k_alpha_split_zero, dim3(blocks_for(nnz)), dim3(TPB), 0, st, nnz, layer, L,
                           sp_inst, sp_layer, sp_j, galpha, ga_ld, ga_off);
    return hipGetLastError();
}

hipError_t launch_prep_splits(const NetShapes &ns, int used, int n_inst, long n_relu,
                              const float *lo, const float *hi, const int32_t *bound_of,
                              const int32_t *off, const int32_t *idx, const int8_t *sign,
                              Relax *tab, int32_t *infeas, int32_t *sp_inst, int32_t *sp_layer,
                              int32_t *sp_j, int32_t *sp_dup, int n_bounds, int stop_m,
                              int stop_relu, float *stop_cen, float *stop_rad, hipStream_t st) {
    const long T = used > 0 ? ns.l[used - 1].off + ns.l[used - 1].d : 0;
    hipLaunchKernelGGL(k_prep_splits, dim3(blocks_for(n_inst, 64)), dim3(64), 0, st, ns.dev, used, T,
                       n_inst, n_relu, lo, hi, bound_of, off, idx, sign, tab, infeas, sp_inst,
                       sp_layer, sp_j, sp_dup, n_bounds, stop_m, stop_relu, stop_cen, stop_rad);
    return hipGetLastError();
}

hipError_t launch_prep_box(int n_inst, int C0, int HW0, const float *x_lo, const float *x_hi,
                           float *cen, float *rad, hipStream_t st) {
    const long d0 = (long)C0 * HW0, total = d0 * n_inst;
    if (total < 0x7fffffffL)
        hipLaunchKernelGGL(k_prep_box<unsigned>, dim3(blocks_for(total)), dim3(TPB), 0, st, total,
                           d0, C0, HW0, x_lo, x_hi, cen, rad);
    else
        hipLaunchKernelGGL(k_prep_box<long>, dim3(blocks_for(total)), dim3(TPB), 0, st, total, d0,
                           C0, HW0, x_lo, x_hi, cen, rad);
    return hipGetLastError();
}

hipError_t launch_init_spec(long img0, long n_img, int rows, int rpi, const float *spec, long dk,
                            int Ck, int HWk, const float *bias_k, float *lam, float *s,
                            float *mag, float *low, hipStream_t st) {
    hipLaunchKernelGGL(k_init_spec, dim3(blocks_for(n_img * dk)), dim3(TPB), 0, st, img0, n_img,
                       rows, rpi, spec, dk, Ck, HWk, lam);
    hipLaunchKernelGGL(k_init_spec_acc, dim3((unsigned)n_img), dim3(TPB), 0, st, img0, n_img, rows,
                       rpi, spec, dk, HWk, bias_k, s, mag, low);
    return hipGetLastError();
}

hipError_t launch_init_identity(const IdentityParams &p, long n_img, bool conc, hipStream_t st) {
    if (conc)
        hipLaunchKernelGGL(k_init_identity<true>, dim3((unsigned)n_img), dim3(TPB), 0, st, p, n_img);
    else
        hipLaunchKernelGGL(k_init_identity<false>, dim3((unsigned)n_img), dim3(TPB), 0, st, p, n_img);
    return hipGetLastError();
}

hipError_t launch_beta_sum(int nnz, int rows, const int32_t *off, const int32_t *idx,
                           const int8_t *sign, const int32_t *sp_inst, const int32_t *sp_layer,
                           const int32_t *sp_dup, const float *beta, float *bsum, hipStream_t st) {
    const long total = (long)nnz * rows;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_beta_sum, dim3(blocks_for(total)), dim3(TPB), 0, st, nnz, rows, off, idx,
                       sign, sp_inst, sp_layer, sp_dup, beta, bsum);
    return hipGetLastError();
}

hipError_t launch_finalize(long img0, long n_img, int rows, int rpi, const float *s,
                           const float *low, const float *mag, const int32_t *infeas, bool slack,
                           float *lower, float *upper, long ld, float *offset, float *offset_mag,
                           float *best, float *best_upper, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n_img)), dim3(TPB), 0, st, img0, n_img, rows,
                       rpi, s, low, mag, infeas, slack ? 1 : 0, lower, upper, ld, offset,
                       offset_mag, best, best_upper);
    return hipGetLastError();
}

hipError_t launch_adj_init(long n_img, int rows, long d0, const float *gl, const float *g1,
                           const float *cen, const float *rad, const int32_t *infeas, float *gbar,
                           float *sbar, hipStream_t st) {
    const long total = n_img * d0;
    const bool al16 = (((uintptr_t)g1 | (uintptr_t)cen | (uintptr_t)rad | (uintptr_t)gbar) & 15) == 0;
    if (d0 % 4 == 0 && al16 && total / 4 < 0x7fffffffL)
        hipLaunchKernelGGL(k_adj_init4, dim3(blocks_for(total / 4)), dim3(TPB), 0, st, n_img, rows,
                           d0, gl, g1, cen, rad, infeas, gbar, sbar);
    else
        hipLaunchKernelGGL(k_adj_init, dim3(blocks_for(total)), dim3(TPB), 0, st, n_img, rows, d0,
                           gl, g1, cen, rad, infeas, gbar, sbar);
    return hipGetLastError();
}

hipError_t launch_beta_grad(int nnz, int rows, int layer, const BetaGradLayer &L,
                            const int32_t *sp_inst, const int32_t *sp_layer, const int32_t *sp_j,
                            const int32_t *sp_dup, const int8_t *sign, const float *gbar_m,
                            const float *sbar, const int32_t *, float *gbeta, hipStream_t st) {
    const long waves = nnz;
    if (waves == 0 || rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_beta_grad, dim3(blocks_for(waves * 64)), dim3(TPB), 0, st, nnz, rows,
                       layer, L, sp_inst, sp_layer, sp_j, sp_dup, sign, gbar_m, sbar, gbeta);
    return hipGetLastError();
}

hipError_t launch_prep_stop_box(int n_inst, const LayerShape &L, long n_relu, const float *lo,
                                const float *hi, const int32_t *bound_of, int n_bounds, bool relu,
                                float *cen, float *rad, hipStream_t st) {
    const long total = (long)n_inst * L.d;
    hipLaunchKernelGGL(k_prep_stop_box, dim3(blocks_for(total)), dim3(TPB), 0, st, total, L, n_relu,
                       lo, hi, bound_of, n_bounds, relu ? 1 : 0, cen, rad);
    return hipGetLastError();
}

hipError_t launch_box_conc(long img0, long n_img, int rpi, long D, const float *lam, const float *cen,
                           const float *rad, float *low, float *mag, float *save, hipStream_t st) {
    if (n_img <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_box_conc, dim3((unsigned)n_img), dim3(TPB), 0, st, img0, rpi, D, lam, cen,
                       rad, low, mag, save);
    return hipGetLastError();
}

hipError_t launch_adj_stop_linear(long n_img, int rows, long D, const float *lam, const float *g,
                                  const float *cen, const float *rad, const float *gl,
                                  const int32_t *infeas, float *sbar, const Relax *tab, long tab_ld,
                                  float *gout, float *gc, int C, int HW, hipStream_t st) {
    const long total = n_img * D;
    hipLaunchKernelGGL(k_adj_stop_linear, dim3(blocks_for(total)), dim3(TPB), 0, st, n_img, rows, D,
                       lam, g, cen, rad, gl, infeas, sbar, tab, tab_ld, gout, gc, C, HW);
    return hipGetLastError();
}

hipError_t launch_beta_grad_stop(int nnz, int rows, int layer, long D, const int32_t *sp_inst,
                                 const int32_t *sp_layer, const int32_t *sp_j, const int8_t *sign,
                                 const float *lam, const float *cen, const float *rad,
                                 const float *sbar, float *gbeta, hipStream_t st) {
    const long total = (long)nnz * rows;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_beta_grad_stop, dim3(blocks_for(total)), dim3(TPB), 0, st, nnz, rows, layer,
                       D, sp_inst, sp_layer, sp_j, sign, lam, cen, rad, sbar, gbeta);
    return hipGetLastError();
}

hipError_t launch_to_internal(long n_img, int C, int HW, const float *x, float *y, hipStream_t st) {
    const long D = (long)C * HW, total = n_img * D;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_internal, dim3(blocks_for(total)), dim3(TPB), 0, st, total, D, C, HW, x, y);
    return hipGetLastError();
}

hipError_t launch_sample_minmax(long n_sub, int per_sub, long D, int C, int HW, float *z, float *lo,
                                float *hi, long ld, bool relu, float *out, bool merge, hipStream_t st) {
    const long total = n_sub * D;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample_minmax, dim3(blocks_for(total)), dim3(TPB), 0, st, n_sub, per_sub, D,
                       C, HW, z, lo, hi, ld, relu ? 1 : 0, out, merge ? 1 : 0);
    return hipGetLastError();
}

AdamArgs adam_args(int step, float lr, float b1, float b2, float eps, float gs, float lo, float hi) {
    AdamArgs a;
    a.b1 = b1;
    a.b2 = b2;
    a.bc1 = 1.f - powf(b1, (float)step);
    a.bc2s = sqrtf(1.f - powf(b2, (float)step));
    a.lr = lr;
    a.eps = eps;
    a.gs = gs;
    a.lo = lo;
    a.hi = hi;
    return a;
}

hipError_t launch_adam(long n, float *p, const float *g, float *m, float *v, int step, float lr,
                       float b1, float b2, float eps, float gs, float lo, float hi, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(TPB), 0, st, n, p, g, m, v,
                       adam_args(step, lr, b1, b2, eps, gs, lo, hi));
    return hipGetLastError();
}

hipError_t launch_alpha_adam(int n_inst, int rows, long D, const LayerShape &L, int layer,
                             long n_relu, const int32_t *srow, const int32_t *slot_count,
                             const int32_t *slot_inv, const int32_t *slot, float *gc, float *alpha,
                             float *m, float *v, long ld, long aoff, int nnz,
                             const int32_t *sp_inst, const int32_t *sp_layer, const int32_t *sp_j,
                             const AdamArgs &a, hipStream_t st) {
    if (n_inst <= 0 || D <= 0) return hipSuccess;
    if (nnz > 0) {
        const long nt = (long)nnz * rows;
        hipLaunchKernelGGL(k_split_gc_zero, dim3(blocks_for(nt)), dim3(TPB), 0, st, nnz, rows, layer,
                           D, n_relu, (long)L.off, sp_inst, sp_layer, sp_j, srow, slot, gc);
    }
    hipLaunchKernelGGL(k_alpha_adam, dim3((unsigned)n_inst), dim3(TPB), 0, st, rows, D, L, layer,
                       n_relu, srow, slot_count, slot_inv, gc, alpha, m, v, ld, aoff, a);
    return hipGetLastError();
}

hipError_t launch_concretize(int n_inst, int rows, long d0, const float *coeff,
                             const float *offset, const float *offset_mag, const float *x_lo,
                             const float *x_hi, bool slack, float *lower, hipStream_t st) {
    const long nrow = (long)n_inst * rows;
    if (nrow == 0) return hipSuccess;
    hipLaunchKernelGGL(k_concretize, dim3((unsigned)n_inst), dim3(TPB), 0, st, rows, d0, coeff,
                       offset, offset_mag, x_lo, x_hi, slack ? 1 : 0, lower);
    return hipGetLastError();
}

hipError_t launch_pack_T(const float *W, int kind, int ci, int hi_, int wi, int co, int ho, int wo,
                         int kh, int kw, int stride, int pad, int py, int px, int ky0, int kx0,
                         int Ty, int Tx, int N, int K, int Kp, int Np, float *Bt, hipStream_t st) {
    (void)ho; (void)wo; (void)pad; (void)py; (void)px;
    const long total = (long)Np * Kp;
    hipLaunchKernelGGL(k_pack_T, dim3(blocks_for(total)), dim3(TPB), 0, st, W, kind, ci, hi_ * wi,
                       co, kh, kw, stride, ky0, kx0, Ty, Tx, N, K, Kp, total, Bt);
    return hipGetLastError();
}

hipError_t launch_pack_F(const float *W, int kind, int ci, int hi_, int wi, int co, int kh, int kw,
                         int N, int K, int Kp, int Np, float *Bt, hipStream_t st) {
    (void)co;
    const long total = (long)Np * Kp;
    hipLaunchKernelGGL(k_pack_F, dim3(blocks_for(total)), dim3(TPB), 0, st, W, kind, ci, hi_ * wi,
                       kh, kw, N, K, Kp, total, Bt);
    return hipGetLastError();
}

}  // namespace bp
