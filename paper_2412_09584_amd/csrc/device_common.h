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

// ---------------------------------------------------------------------- epilogues
struct EpiRelax {
    RelaxParams p;
    static constexpr int NRED = 2;
    struct Row { long inst; };
    __device__ Row row(long img) const { return Row{(p.img0 + img) / p.rpi}; }
    __device__ float colv(int n) const { return p.bias[n % p.chan]; }
    __device__ float *red0() const { return p.s; }
    __device__ float *red1() const { return p.mag; }
    __device__ void elem(const Row &rc, long img, long dpix, int n, long j, float bcol, float g,
                         float &r0, float &r1) const {
        const Relax t = p.tab[rc.inst * p.tab_ld + j];
        const float lam = g >= 0.f ? g * t.x : g * t.y;
        const float off = g < 0.f ? g * t.z : 0.f;
        const float bt = lam * bcol;
        r0 += bt + off;
        r1 += fabsf(bt) + fabsf(off);
        const long o = img * p.D + j;
        p.out[o] = lam;
        if (p.save) p.save[o] = g;
    }
};

struct EpiConc {
    ConcParams p;
    static constexpr int NRED = 2;
    struct Row { long inst; };
    __device__ Row row(long img) const { return Row{(p.img0 + img) / p.rpi}; }
    __device__ float colv(int) const { return 0.f; }
    __device__ float *red0() const { return p.low; }
    __device__ float *red1() const { return p.mag; }
    __device__ void elem(const Row &rc, long img, long dpix, int n, long j, float, float g,
                         float &r0, float &r1) const {
        const long ij = rc.inst * p.D + j;
        const float c = p.cen[ij], r = p.rad[ij];
        r0 += g * c - fabsf(g) * r;
        r1 += fabsf(g) * (fabsf(c) + r);
        if (p.save) p.save[img * p.D + j] = g;
        if (p.emit) p.emit[img * p.D + (long)n * p.hw + dpix] = g;
    }
};

struct EpiAdj {
    AdjParams p;
    static constexpr int NRED = 0;
    struct Row { long inst; float sb; };
    __device__ Row row(long img) const { return Row{img / p.rpi, p.sbar[img]}; }
    __device__ float colv(int n) const { return p.bias[n]; }
    __device__ float *red0() const { return nullptr; }
    __device__ float *red1() const { return nullptr; }
    __device__ void elem(const Row &rc, long img, long dpix, int n, long j, float bcol, float acc,
                         float &, float &) const {
        const float v = acc + rc.sb * bcol;           // Lambda_bar_m[img, j]
        const long o = img * p.D + j;
        const float g = p.gsave[o];                   // G_{m+1}[img, j]
        const Relax t = p.tab[rc.inst * p.tab_ld + j];
        if (p.gout) p.gout[o] = v * (g >= 0.f ? t.x : t.y) + (g < 0.f ? rc.sb * t.z : 0.f);
        if (t.w != 0.f && g >= 0.f) {
            const float c = g * v;
            if (c != 0.f) atomicAdd(p.galpha + rc.inst * p.ga_ld + p.ga_off + (long)n * p.hw + dpix, c);
        }
    }
};

// Forward pass of sample rows (search-integrated bounds): z = W h + b.
struct EpiFwd {
    FwdParams p;
    static constexpr int NRED = 0;
    struct Row {};
    __device__ Row row(long) const { return Row{}; }
    __device__ float colv(int n) const { return p.bias[n]; }
    __device__ float *red0() const { return nullptr; }
    __device__ float *red1() const { return nullptr; }
    __device__ void elem(const Row &, long img, long, int, long j, float bcol, float acc, float &,
                         float &) const {
        p.out[img * p.D + j] = acc + bcol;
    }
};

// Sum of r0 / r1 over the lanes that hold the same output row (they differ only in the
// column bits of the lane id), then one atomic per row from the column-0 lane.
template <int MF>
__device__ inline void reduce_row_atomic(float r0, float r1, long img, int lane, float *red0,
                                         float *red1) {
#pragma unroll
    for (int mk = 1; mk < MF; mk <<= 1) {
        r0 += __shfl_xor(r0, mk, 64);
        r1 += __shfl_xor(r1, mk, 64);
    }
    if ((lane & (MF - 1)) == 0 && img >= 0) {
        atomicAdd(red0 + img, r0);
        atomicAdd(red1 + img, r1);
    }
}

__device__ inline void reduce_wave_atomic(float u0, float u1, long img, int lane, float *red0,
                                          float *red1) {
#pragma unroll
    for (int mk = 1; mk < 64; mk <<= 1) {
        u0 += __shfl_xor(u0, mk, 64);
        u1 += __shfl_xor(u1, mk, 64);
    }
    if (lane == 0) {
        atomicAdd(red0 + img, u0);
        atomicAdd(red1 + img, u1);
    }
}

}  // namespace dev
}  // namespace bp
