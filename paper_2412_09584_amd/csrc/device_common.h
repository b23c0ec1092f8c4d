// Device code shared by the gfx950 product kernels: MFMA lane layouts and the fused
// epilogues of the bound pass (Lemma 1 relaxation, Theorem 2 concretisation) and of
// its adjoint.
#pragma once
#include "bound_internal.h"

namespace bp {
namespace dev {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

template <int MF> struct Mma;
template <> struct Mma<32> {
    using acc_t = f32x16;
    static constexpr int NACC = 16;
    static constexpr int KPL = 8;  // k values per lane per chunk (2 lane groups)
    static __device__ inline acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }
    static __device__ inline int col(int lane) { return lane & 31; }
    static __device__ inline int grp(int lane) { return lane >> 5; }
    static __device__ inline int idx(int lane) { return lane & 31; }
};
template <> struct Mma<16> {
    using acc_t = f32x4v;
    static constexpr int NACC = 4;
    static constexpr int KPL = 4;  // 4 lane groups
    static __device__ inline acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int v, int lane) { return 4 * (lane >> 4) + v; }
    static __device__ inline int col(int lane) { return lane & 15; }
    static __device__ inline int grp(int lane) { return lane >> 4; }
    static __device__ inline int idx(int lane) { return lane & 15; }
};

// ---------------------------------------------------------------------- tile order
// Logical tile (x, y, z) of this workgroup in an [nx][ny][nz] tile grid launched as a
// one-dimensional grid of nx * ny * nz workgroups.  Workgroups are dispatched to the 8
// XCDs round-robin (workgroup b to XCD b mod 8) and every XCD has its own L2, so the
// renumbering hands XCD k the k-th contiguous range of logical tiles, z (the output
// phase of a transposed convolution) fastest and y (the column tile) next: tiles that
// gather the same input rows, and the rows of one instance, which share its relaxation
// records, then meet in one L2 at about the same time.
struct TileIdx {
    long x;
    int y, z;
};
__device__ inline TileIdx xcd_tile(int ny, int nz) {
    const unsigned T = gridDim.x, b = blockIdx.x;
    const unsigned q = T >> 3, r = T & 7, xcd = b & 7, slot = b >> 3;
    unsigned t = xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
    TileIdx ti;
    ti.z = (int)(t % (unsigned)nz);
    t /= (unsigned)nz;
    ti.y = (int)(t % (unsigned)ny);
    ti.x = (long)(t / (unsigned)ny);
    return ti;
}

// ---------------------------------------------------------------------- index helpers
// n / d for 0 <= n < 2^21 through one FP32 multiply by rd = fl(1/d): (n + 0.5) / d lies
// at least 0.5/d away from an integer, and the two roundings move the product by less
// than (n + 0.5)/d * 2^-23 < 0.5/d, so truncation gives the exact quotient.
__device__ inline int qdiv(int n, float rd) { return (int)(((float)n + 0.5f) * rd); }
__device__ inline long ldiv_by(long n, int d, float rd) {
    return n < (1L << 21) ? (long)qdiv((int)n, rd) : n / d;
}
// The same in FP64 with rd = fl64(1 / d): exact for 0 <= n < 2^50 by the argument above
// with 2^-52 in place of 2^-23.
__device__ inline long ldiv64(long n, double rd) { return (long)(((double)n + 0.5) * rd); }

// Element i of one img's row segment starting at base.  Every epilogue offset stays inside
// such a segment (i * sizeof(T) < 2^32, layer widths are validated on the host), so the
// byte offset is formed in 32 bits; the access goes through a global-address-space
// pointer, so that with a wave-uniform base it takes the scalar-base global form (a
// generic pointer that the compiler cannot place would give a flat access with 64-bit
// address arithmetic per element).
template <class T> __device__ inline T ld(const T *base, int i) {
    using G = const __attribute__((address_space(1))) T;
    return *(G *)((const char *)base + (unsigned)i * (unsigned)sizeof(T));
}
// float4 records through the compiler's native vector type (HIP's float4 class has no
// copy from another address space)
__device__ inline float4 ld(const float4 *base, int i) {
    using V = float __attribute__((ext_vector_type(4)));
    using G = const __attribute__((address_space(1))) V;
    const V v = *(G *)((const char *)base + (unsigned)i * 16u);
    return make_float4(v.x, v.y, v.z, v.w);
}
template <class T> __device__ inline void st(T *base, int i, T v) {
    using G = __attribute__((address_space(1))) T;
    *(G *)((char *)base + (unsigned)i * (unsigned)sizeof(T)) = v;
}

// ---------------------------------------------------------------------- LDS DMA
// dword 3 of a raw buffer resource (32-bit data format; no swizzle, no index stride)
constexpr int BUF_FLAGS = 0x00020000;

// 16 bytes per lane from base + voff (bytes) into LDS at lds + 16 * lane (lds uniform
// across the wave); offsets at or past nbytes read nothing.
__device__ inline void lds_dma16(const float *base, int nbytes, float *lds, int voff) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, nbytes, BUF_FLAGS);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void *)lds, 16,
                                             voff, 0, 0, 0);
}

// ---------------------------------------------------------------------- epilogues
// Each epilogue splits its per-element work into pre() -- the global loads it needs
// (relaxation record, box) --, pre2() -- loads whose address depends on pre()'s result
// (the saved coefficient of the adjoint) -- and post() -- arithmetic, stores and
// atomics -- so that tile_epilogue can issue loads ahead of earlier groups' stores.
// Row(img) resolves the per-img pointers once per row group; j is the element's offset
// inside its img (dpix * N + n), dpix the destination pixel.
struct EpiRelax {
    RelaxParams p;
    static constexpr int NRED = 2;
    using Pre = Relax;
    struct Row { const Relax *tb; float *out, *save; };
    __device__ Row row(int img) const {
        const long inst = ldiv_by(p.img0 + img, p.rpi, p.rrpi);
        const long o = (long)img * p.D;
        return Row{p.tab + inst * p.tab_ld, p.out + o, p.save ? p.save + o : nullptr};
    }
    // split multipliers' term of row rc at first split entry q: the row within its
    // instance is recovered from the row's output pointer (only on this rare path, so the
    // common path keeps no extra register per row)
    __device__ float split_term(const Row &rc, int q) const {
        const long gi = p.img0 + (rc.out - p.out) / p.D;
        const long r = gi - (gi / p.rpi) * p.rpi;
        return p.bsum[(long)q * p.rpi + r];
    }
    __device__ float colv(int n) const { return p.bias[n % p.chan]; }
    __device__ float *red0() const { return p.s; }
    __device__ float *red1() const { return p.mag; }
    __device__ const DetSums *det() const { return &p.det; }
    __device__ Pre pre(const Row &rc, int j) const { return ld(rc.tb, j); }
    __device__ void pre2(const Row &, Pre &) const {}
    __device__ void post(const Pre &t, const Row &rc, int, int, int j, float bcol, float g,
                         float &r0, float &r1) const {
        // Lemma 1's line by the sign of G, then -sum(beta sign) of the split entries at a
        // split neuron (first entry q = -w - 1); split neurons are a few per instance, so
        // their term is loaded here, in a branch most waves skip, rather than carried in
        // registers with every element's record.  The bias term takes the coefficient with
        // the split term included.
        float lam = g >= 0.f ? g * t.x : g * t.y;
        if (t.w < 0.f && p.bsum) lam -= split_term(rc, -(int)t.w - 1);
        const float off = g < 0.f ? g * t.z : 0.f;
        const float bt = lam * bcol;
        r0 += bt + off;
        r1 += fabsf(bt) + fabsf(off);
        // the sums are formed in order; without this the compiler defers them past the
        // tile's stores and keeps every lam and offset of the tile live in registers
        asm volatile("" : "+v"(r0), "+v"(r1));
        st(rc.out, j, lam);
        if (rc.save && t.w > 0.f) st(rc.save, (int)t.w - 1, g);    // unstable: compact slot
    }
};

struct EpiConc {
    ConcParams p;
    static constexpr int NRED = 2;
    using Pre = float2;
    struct Row { const float *cen, *rad; float *save, *emit; };
    __device__ Row row(int img) const {
        const long inst = ldiv_by(p.img0 + img, p.rpi, p.rrpi);
        const long o = (long)img * p.D;
        return Row{p.cen + inst * p.D, p.rad + inst * p.D, p.save ? p.save + o : nullptr,
                   p.emit ? p.emit + o : nullptr};
    }
    __device__ float colv(int) const { return 0.f; }
    __device__ float *red0() const { return p.low; }
    __device__ float *red1() const { return p.mag; }
    __device__ const DetSums *det() const { return &p.det; }
    __device__ Pre pre(const Row &rc, int j) const { return make_float2(ld(rc.cen, j), ld(rc.rad, j)); }
    __device__ void pre2(const Row &, Pre &) const {}
    __device__ void post(const Pre &cr, const Row &rc, int dpix, int n, int j, float, float g,
                         float &r0, float &r1) const {
        r0 += g * cr.x - fabsf(g) * cr.y;
        r1 += fabsf(g) * (fabsf(cr.x) + cr.y);
        asm volatile("" : "+v"(r0), "+v"(r1));   // in order, as in EpiRelax
        if (rc.save) st(rc.save, j, g);
        if (rc.emit) st(rc.emit, n * p.hw + dpix, g);
    }
};

struct EpiAdj {
    AdjParams p;
    static constexpr int NRED = 0;
    struct Pre { Relax t; float g; };
    struct Row { const Relax *tb; const float *gs; float *go; float *gc; float *gb; float sb; };
    __device__ Row row(int img) const {
        const long inst = ldiv_by(img, p.rpi, p.rrpi);
        const long o = (long)img * p.D;
        return Row{p.tab + inst * p.tab_ld, p.gsave + o, p.gout ? p.gout + o : nullptr,
                   p.gc + o, p.gbeta ? p.gbeta + (img - inst * p.rpi) : nullptr, p.sbar[img]};
    }
    __device__ float colv(int n) const { return p.bias[n]; }
    __device__ float *red0() const { return nullptr; }
    __device__ float *red1() const { return nullptr; }
    __device__ const DetSums *det() const { return nullptr; }
    // G is saved at the unstable neurons only (slot w - 1), a load that depends on the
    // record: pre() fetches the record, pre2() the saved coefficient.  Elsewhere x = y
    // and z = 0, so the sign of G does not matter.
    __device__ Pre pre(const Row &rc, int j) const { return Pre{ld(rc.tb, j), 0.f}; }
    __device__ void pre2(const Row &rc, Pre &q) const {
        if (q.t.w > 0.f) q.g = ld(rc.gs, (int)q.t.w - 1);
    }
    __device__ void post(const Pre &q, const Row &rc, int dpix, int n, int j, float bcol, float acc,
                         float &, float &) const {
        const float v = acc + rc.sb * bcol;           // Lambda_bar_m[img, j]
        const float g = q.g;                          // G_{m+1}[img, j]
        const Relax &t = q.t;
        if (rc.go) st(rc.go, j, v * (g >= 0.f ? t.x : t.y) + (g < 0.f ? rc.sb * t.z : 0.f));
        // alpha-gradient contribution of this row at the neuron's slot (summed over the
        // instance's rows by k_alpha_grad)
        if (t.w > 0.f) st(rc.gc, (int)t.w - 1, g >= 0.f ? g * v : 0.f);
        // split neuron (first entry q of the instance's list): d lower / d beta_{q,r} =
        // -sign_q * Lambda_bar, sign_q carried in the sign bit of the record's z
        if (t.w < 0.f && rc.gb) rc.gb[(long)(-(int)t.w - 1) * p.rpi] = signbit(t.z) ? v : -v;
    }
};

// Forward pass of sample rows (search-integrated bounds): z = W h + b.
struct EpiFwd {
    FwdParams p;
    static constexpr int NRED = 0;
    struct Pre {};
    struct Row { float *out; };
    __device__ Row row(int img) const { return Row{p.out + (long)img * p.D}; }
    __device__ float colv(int n) const { return p.bias[n]; }
    __device__ float *red0() const { return nullptr; }
    __device__ float *red1() const { return nullptr; }
    __device__ const DetSums *det() const { return nullptr; }
    __device__ Pre pre(const Row &, int) const { return Pre{}; }
    __device__ void pre2(const Row &, Pre &) const {}
    __device__ void post(const Pre &, const Row &rc, int, int, int j, float bcol, float acc,
                         float &, float &) const {
        st(rc.out, j, acc + bcol);
    }
};

// One row sum pair of a tile: a float atomic per accumulator, or with deterministic sums
// a store to the tile's own slot (dp: destination pixel of the tile's first row, n0: its
// first column).
template <class Epi>
__device__ inline void put_row_sums(const Epi &epi, long img, int dp, int n0, float r0, float r1) {
    const DetSums *d = epi.det();
    if (d && d->part) {
        float *q = d->part + (img * d->nslot + (long)dp * d->ncu + (n0 >> 4)) * 2;
        q[0] = r0;
        q[1] = r1;
    } else {
        atomicAdd(epi.red0() + img, r0);
        atomicAdd(epi.red1() + img, r1);
    }
}

// Sum of r0 / r1 over the lanes that hold the same output row (they differ only in the
// column bits of the lane id), then one sum pair per row from the column-0 lane.
template <int MF, class Epi>
__device__ inline void reduce_row(const Epi &epi, float r0, float r1, int img, int dp, int n0,
                                  int lane) {
#pragma unroll
    for (int mk = 1; mk < MF; mk <<= 1) {
        r0 += __shfl_xor(r0, mk, 64);
        r1 += __shfl_xor(r1, mk, 64);
    }
    if ((lane & (MF - 1)) == 0 && img >= 0) put_row_sums(epi, img, dp, n0, r0, r1);
}

// The sums of a whole wave (one img), then one pair from lane 0 (which holds the wave's
// first row and its tile's first column).
template <class Epi>
__device__ inline void reduce_wave(const Epi &epi, float u0, float u1, long img, int dp, int n0,
                                   int lane) {
#pragma unroll
    for (int mk = 1; mk < 64; mk <<= 1) {
        u0 += __shfl_xor(u0, mk, 64);
        u1 += __shfl_xor(u1, mk, 64);
    }
    if (lane == 0) put_row_sums(epi, img, dp, n0, u0, u1);
}

// Epilogue of one wave's accumulator tile.  The accumulator rows of a lane come in
// groups of four consecutive tile rows (MFMA row groups); rowfn4(i, vg, img, dp) maps
// group vg of fragment i to the local img of each row (-1 if out of range) and its
// destination pixel, and returns true when all four rows lie in one img (then the
// per-img pointers are resolved once).  A group's loads are issued before its stores.
// FAST: every row of the wave lies in img uimg and every column is in range (the
// common case of a convolution tile), so the pointers are resolved once per wave, no
// element is masked and the row sums collapse into one atomic pair per wave.
template <bool FAST, bool LEAN, class Epi, int MF, int FM, int FN, class Acc, class RowFn>
__device__ inline void tile_epilogue_impl(const Epi &epi, Acc (&acc)[FM][FN], const int (&ncol)[FN],
                                          const float (&bcol)[FN], int N, const RowFn &rowfn4,
                                          int lane, int uimg) {
    constexpr int NACC = Mma<MF>::NACC;
    constexpr int NR = Epi::NRED;
    float u0 = 0.f, u1 = 0.f;
    typename Epi::Row rw;
    if (FAST) {
        // Pipeline over the row groups: the first loads of group g + 2 and the dependent
        // loads of group g + 1 are issued before the stores of group g (records and saved
        // coefficients never alias the outputs), so about one memory latency is exposed
        // per tile rather than one or two per group -- when three groups' loads fit in
        // about 64 registers (else two stages, or none).
        rw = epi.row(__builtin_amdgcn_readfirstlane(uimg));
        constexpr int NG = FM * (NACC / 4);
        constexpr int GREG = FN * 4 * (int)sizeof(typename Epi::Pre) / 4;
        constexpr int DEPTH = 2 * GREG <= 48 ? 1 : 0;
        using PreG = typename Epi::Pre[FN][4];
        auto load1 = [&](int g, int (&dp)[4], PreG &pre) {
            int img[4];
            rowfn4(g / (NACC / 4), g % (NACC / 4), img, dp);
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) pre[j][q] = epi.pre(rw, dp[q] * N + ncol[j]);
        };
        auto load2 = [&](PreG &pre) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) epi.pre2(rw, pre[j][q]);
        };
        auto copy = [&](int (&dd)[4], PreG &pd, const int (&ds)[4], const PreG &ps) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                dd[q] = ds[q];
#pragma unroll
                for (int j = 0; j < FN; ++j) pd[j][q] = ps[j][q];
            }
        };
        int dpA[4], dpB[4];
        PreG preA, preB;
        load1(0, dpA, preA);
        load2(preA);
        const int dp0 = dpA[0];           // lane 0: the wave's first row
        if (DEPTH == 2 && NG > 1) load1(1, dpB, preB);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            int dpC[4];
            PreG preC;
            if (DEPTH == 2) {
                if (g + 2 < NG) load1(g + 2, dpC, preC);
                if (g + 1 < NG) load2(preB);
            } else if (DEPTH == 1 && g + 1 < NG) {
                load1(g + 1, dpB, preB);
                load2(preB);
            }
            const int i = g / (NACC / 4), vg = g % (NACC / 4);
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    epi.post(preA[j][q], rw, dpA[q], ncol[j], dpA[q] * N + ncol[j], bcol[j],
                             acc[i][j][vg * 4 + q], u0, u1);
            if (DEPTH == 0 && g + 1 < NG) {
                load1(g + 1, dpB, preB);
                load2(preB);
            }
            if (g + 1 < NG) copy(dpA, preA, dpB, preB);
            if (DEPTH == 2 && g + 2 < NG) copy(dpB, preB, dpC, preC);
        }
        if (NR > 0) reduce_wave(epi, u0, u1, uimg, dp0, ncol[0], lane);
        return;
    }
    if (LEAN) {
        // one element at a time: the rare tiles of a convolution that straddle images
        // or the end of the batch; few registers, so the common path keeps its occupancy
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
            for (int vg = 0; vg < NACC / 4; ++vg) {
                int img[4], dp[4];
                rowfn4(i, vg, img, dp);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float r0 = 0.f, r1 = 0.f;
                    if (img[q] >= 0) {
                        const typename Epi::Row rc = epi.row(img[q]);
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            if (ncol[j] < N) {
                                typename Epi::Pre pr = epi.pre(rc, dp[q] * N + ncol[j]);
                                epi.pre2(rc, pr);
                                epi.post(pr, rc, dp[q], ncol[j], dp[q] * N + ncol[j], bcol[j],
                                         acc[i][j][vg * 4 + q], r0, r1);
                            }
                    }
                    if (NR > 0) reduce_row<MF>(epi, r0, r1, img[q], dp[q], ncol[0], lane);
                }
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int vg = 0; vg < NACC / 4; ++vg) {
            int img[4], dp[4];
            typename Epi::Row rc[4];
            const bool one = rowfn4(i, vg, img, dp);
            if (FAST) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    img[q] = uimg;
                    rc[q] = rw;
                }
            } else if (one) {
                if (img[0] >= 0) rc[0] = epi.row(img[0]);
                rc[1] = rc[2] = rc[3] = rc[0];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (img[q] >= 0) rc[q] = epi.row(img[q]);
            }
            float r0[4] = {0.f, 0.f, 0.f, 0.f}, r1[4] = {0.f, 0.f, 0.f, 0.f};
            typename Epi::Pre pre[FN][4];
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (FAST || (img[q] >= 0 && ncol[j] < N)) {
                        pre[j][q] = epi.pre(rc[q], dp[q] * N + ncol[j]);
                        epi.pre2(rc[q], pre[j][q]);
                    }
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (FAST || (img[q] >= 0 && ncol[j] < N))
                        epi.post(pre[j][q], rc[q], dp[q], ncol[j], dp[q] * N + ncol[j], bcol[j],
                                 acc[i][j][vg * 4 + q], FAST ? u0 : r0[q], FAST ? u1 : r1[q]);
            if (NR > 0 && !FAST) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    reduce_row<MF>(epi, r0[q], r1[q], img[q], dp[q], ncol[0], lane);
            }
        }
    }
}

// fast: see tile_epilogue_impl (wave-uniform).
// LEAN: the other tiles take the one-element-at-a-time path (convolution tiles, where
// they are rare) instead of the batched one (dense products, where every tile is such).
template <class Epi, int MF, int FM, int FN, bool LEAN = false, class Acc, class RowFn>
__device__ inline void tile_epilogue(const Epi &epi, Acc (&acc)[FM][FN], const int (&ncol)[FN],
                                     const float (&bcol)[FN], int N, const RowFn &rowfn4, int lane,
                                     bool fast, int uimg) {
    if (fast)
        tile_epilogue_impl<true, false, Epi, MF, FM, FN>(epi, acc, ncol, bcol, N, rowfn4, lane, uimg);
    else
        tile_epilogue_impl<false, LEAN, Epi, MF, FM, FN>(epi, acc, ncol, bcol, N, rowfn4, lane, -1);
}

}  // namespace dev
}  // namespace bp
