// FP32 MFMA implicit-GEMM kernels for gfx950 with fused bound-propagation epilogues.
//
// One kernel template covers every product on the bound path:
//  * the backward step of Theorem 1, G_m = Lambda_m W_m (Linear: a dense GEMM; Conv2d:
//    the transposed convolution, run as one stride-1 implicit GEMM per output phase),
//    with Lemma 1's relaxation, the bias / intercept row sums (the offset b~) and the
//    FP32 rounding-allowance magnitudes fused into the epilogue (EpiRelax);
//  * the last step G_1 = Lambda_1 W_1 with Theorem 2's box concretisation fused into the
//    epilogue, so G_1 need not reach HBM (EpiConc);
//  * the adjoint step Lambda_bar_m = G_bar_m W_m^T (Linear) or the forward convolution
//    (Conv2d), with the reverse of the relaxation and the alpha-gradient reduction
//    fused into the epilogue (EpiAdj).
//
// Tiling: 256 threads = 4 wave64s; a block owns a BM x BN output tile; K advances in
// chunks of 16 staged through LDS (A rows and B columns both stored k-contiguous, so a
// lane fetches its k values with 128-bit LDS reads) with the next chunk's global loads
// in flight during the MFMAs.  v_mfma_f32_32x32x2f32 serves N >= 32 and
// v_mfma_f32_16x16x4f32 the narrow N = 16 products.  Within a 16-wide k chunk lane
// group h of the MFMA supplies k = h*KPL + s at step s, which lets each lane read KPL
// consecutive k from LDS.
#include "device_common.h"

namespace bp {
namespace {

constexpr int BK = 16;
constexpr int LDSW = BK + 4;  // LDS row stride in floats (keeps 16-byte alignment)

using namespace dev;

// ---------------------------------------------------------------------- the kernel
// k -> (ky, kx, c) of the implicit-GEMM gather, decoded once per block into LDS:
// .x = offset of (ky, kx, c) from the row's top-left source element, .y = ky << 16 | kx.
constexpr int KDEC_MAX = 1024;

// DMAG (dense products, K a multiple of 16): the k chunks go from global memory straight
// into LDS by DMA, two buffers deep -- chunk k + 1 is in flight while chunk k's MFMAs
// run, one barrier per chunk, no staging registers.  LDS rows are unpadded (16 floats)
// with the four 16-byte k quads of row r stored in the order kq ^ ((r >> 1) & 3), so the
// operand reads of consecutive rows fall in different banks.
template <class Epi, int MF, int BM, int BN, int WGM, int WGN, bool DENSE, bool VEC, bool DMAG = false>
__global__ __launch_bounds__(256) void k_gemm(const GeomSet gs, const float *__restrict__ A,
                                              const long n_img, const Epi epi) {
    static_assert(!DMAG || (DENSE && VEC), "DMA chunks for dense products");
    using MM = Mma<MF>;
    using acc_t = typename MM::acc_t;
    constexpr int TM = BM / WGM, TN = BN / WGN, FM = TM / MF, FN = TN / MF;
    static_assert(WGM * WGN == 4, "4 waves");
    static_assert(FM >= 1 && FN >= 1, "wave tile");
    constexpr int KPL = MM::KPL;
    constexpr int AF4 = BM * BK / 4, BF4 = BN * BK / 4;
    constexpr int APT = (AF4 + 255) / 256, BPT = (BF4 + 255) / 256;
    __shared__ __attribute__((aligned(16))) float As[DMAG ? 2 * BM * BK : BM * LDSW];
    __shared__ __attribute__((aligned(16))) float Bs[DMAG ? 2 * BN * BK : BN * LDSW];
    __shared__ int2 kdec[DENSE ? 1 : KDEC_MAX];

    const TileIdx ti = xcd_tile((gs.g[0].N + BN - 1) / BN, gs.n);
    const Geom &g = gs.g[ti.z];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const long Mimg = (long)g.OH * g.OW;
    const long M = n_img * Mimg;
    const long m0 = ti.x * BM;
    const int n0 = ti.y * BN;
    if (m0 >= M) return;
    const int K = g.K;

    if (!DENSE) {
        for (int k = tid; k < K; k += 256) {
            const int tap = qdiv(k, g.rC), c = k - tap * g.C;
            const int ky = qdiv(tap, g.rKW), kx = tap - ky * g.kw;
            kdec[k] = make_int2((ky * g.W + kx) * g.C + c, (ky << 16) | kx);
        }
        // visible to every thread after the first barrier of the k loop
    }

    // Per-slot source-row state for the A gather (the rows a thread loads never change).
    // Rows are decomposed from the block's first row (one wide division per thread).
    const float *abase[APT];
    int aby[APT], abx[APT], akq[APT], arow[APT];
    bool aok[APT];
    const long bimg = DENSE ? m0 : ldiv64(m0, g.rMd);
    const int bp0 = (int)(m0 - bimg * Mimg);
    const float rMb = g.rM, rOWb = g.rOW;
#pragma unroll
    for (int i = 0; i < APT; ++i) {
        const int f = tid + 256 * i;
        arow[i] = f >> 2;
        akq[i] = (f & 3) * 4;
        const long m = m0 + arow[i];
        aok[i] = (f < AF4) && (m < M);
        abase[i] = A;
        aby[i] = abx[i] = 0;
        if (aok[i]) {
            if (DENSE) {
                abase[i] = A + m * K;
            } else {
                int p = bp0 + arow[i];
                const int kq = qdiv(p, rMb);
                p -= kq * (int)Mimg;
                const long img = bimg + kq;
                const int oy = qdiv(p, rOWb), ox = p - oy * g.OW;
                // top-left source element of this row (may lie outside the image; only
                // in-range elements are ever dereferenced)
                aby[i] = oy * g.stride - g.pad_y;
                abx[i] = ox * g.stride - g.pad_x;
                abase[i] = A + img * (long)g.H * g.W * g.C + ((long)aby[i] * g.W + abx[i]) * g.C;
            }
        }
    }
    const float *bptr[BPT];
    int brow[BPT], bkq[BPT];
    bool bok[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int f = tid + 256 * i;
        brow[i] = f >> 2;
        bkq[i] = (f & 3) * 4;
        bok[i] = f < BF4;
        bptr[i] = g.Bt + (long)(n0 + (bok[i] ? brow[i] : 0)) * g.Kp + bkq[i];
    }

    f32x4v ra[APT], rb[BPT];
    auto gatherA = [&](int i, int k) -> float {
        if (DENSE) return k < K ? abase[i][k] : 0.f;
        if (k >= K) return 0.f;
        const int2 d = kdec[k];
        const int y = aby[i] + (d.y >> 16), x = abx[i] + (d.y & 0xffff);
        if ((unsigned)y >= (unsigned)g.H || (unsigned)x >= (unsigned)g.W) return 0.f;
        return abase[i][d.x];
    };
    auto loadA = [&](int k0) {
#pragma unroll
        for (int i = 0; i < APT; ++i) {
            f32x4v v = {0.f, 0.f, 0.f, 0.f};
            const int k = k0 + akq[i];
            if (aok[i]) {
                if (VEC) {
                    if (DENSE) {
                        if (k < K) v = *(const f32x4v *)(abase[i] + k);
                    } else if (k < K) {
                        const int2 d = kdec[k];
                        const int y = aby[i] + (d.y >> 16), x = abx[i] + (d.y & 0xffff);
                        if ((unsigned)y < (unsigned)g.H && (unsigned)x < (unsigned)g.W)
                            v = *(const f32x4v *)(abase[i] + d.x);
                    }
                } else {
                    v[0] = gatherA(i, k);
                    v[1] = gatherA(i, k + 1);
                    v[2] = gatherA(i, k + 2);
                    v[3] = gatherA(i, k + 3);
                }
            }
            ra[i] = v;
        }
    };
    auto loadB = [&](int k0) {
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            if (bok[i]) rb[i] = *(const f32x4v *)(bptr[i] + k0);
        }
    };

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < MM::NACC; ++v) acc[i][j][v] = 0.f;

    if constexpr (DMAG) {
        constexpr int ASL = BM * BK / 4, BSL = BN * BK / 4;    // float4 slots per buffer
        constexpr int AI = (ASL + 255) / 256, BI = (BSL + 255) / 256;
        auto swz = [](int r, int kq) { return r * 4 + (kq ^ ((r >> 1) & 3)); };
        // slot s = i * 256 + tid of a buffer holds row s / 4, k quad (s & 3) ^ ((r >> 1) & 3)
        int aoff[AI], boff[BI];
#pragma unroll
        for (int i = 0; i < AI; ++i) {
            const int s = i * 256 + tid, r = s >> 2, kq = (s & 3) ^ ((r >> 1) & 3);
            aoff[i] = s < ASL && m0 + r < M ? (r * K + 4 * kq) * 4 : -1;
        }
#pragma unroll
        for (int i = 0; i < BI; ++i) {
            const int s = i * 256 + tid, r = s >> 2, kq = (s & 3) ^ ((r >> 1) & 3);
            boff[i] = s < BSL ? (r * g.Kp + 4 * kq) * 4 : -1;
        }
        const float *Ab = A + m0 * K, *Bb = g.Bt + (long)n0 * g.Kp;
        const int abytes = (int)((M - m0 < BM ? M - m0 : BM) * K * 4), bbytes = BN * g.Kp * 4;
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        auto dma = [&](int k0, int b) {
#pragma unroll
            for (int i = 0; i < AI; ++i)
                if (aoff[i] >= 0) lds_dma16(Ab, abytes, As + b * BM * BK + (i * 256 + wv * 64) * 4, aoff[i] + k0 * 4);
#pragma unroll
            for (int i = 0; i < BI; ++i)
                if (boff[i] >= 0) lds_dma16(Bb, bbytes, Bs + b * BN * BK + (i * 256 + wv * 64) * 4, boff[i] + k0 * 4);
        };
        const int nk = K / BK;
        dma(0, 0);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        for (int kc = 0; kc < nk; ++kc) {
            const int cur = kc & 1;
            if (kc + 1 < nk) dma((kc + 1) * BK, cur ^ 1);
            const float *Ac = As + cur * BM * BK, *Bc = Bs + cur * BN * BK;
            float af[FM][KPL], bf[FN][KPL];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int r = wm * TM + i * MF + MM::idx(lane);
#pragma unroll
                for (int q = 0; q < KPL; q += 4) {
                    const int kq = (MM::grp(lane) * KPL + q) >> 2;
                    const f32x4v t = *(const f32x4v *)(Ac + swz(r, kq) * 4);
                    af[i][q] = t[0]; af[i][q + 1] = t[1]; af[i][q + 2] = t[2]; af[i][q + 3] = t[3];
                }
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int r = wn * TN + j * MF + MM::idx(lane);
#pragma unroll
                for (int q = 0; q < KPL; q += 4) {
                    const int kq = (MM::grp(lane) * KPL + q) >> 2;
                    const f32x4v t = *(const f32x4v *)(Bc + swz(r, kq) * 4);
                    bf[j][q] = t[0]; bf[j][q + 1] = t[1]; bf[j][q + 2] = t[2]; bf[j][q + 3] = t[3];
                }
            }
#pragma unroll
            for (int s = 0; s < KPL; ++s)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = MM::mma(af[i][s], bf[j][s], acc[i][j]);
            // the next chunk has landed, and every wave is done with this one
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
        }
    } else {
    if (!DENSE) __syncthreads();   // decode table complete
    loadA(0);
    loadB(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < APT; ++i)
            if (tid + 256 * i < AF4) *(f32x4v *)(As + arow[i] * LDSW + akq[i]) = ra[i];
#pragma unroll
        for (int i = 0; i < BPT; ++i)
            if (bok[i]) *(f32x4v *)(Bs + brow[i] * LDSW + bkq[i]) = rb[i];
        __syncthreads();
        if (k0 + BK < K) {
            loadA(k0 + BK);
            loadB(k0 + BK);
        }
        float af[FM][KPL], bf[FN][KPL];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const float *src = As + (wm * TM + i * MF + MM::idx(lane)) * LDSW + MM::grp(lane) * KPL;
#pragma unroll
            for (int q = 0; q < KPL; q += 4) {
                const f32x4v t = *(const f32x4v *)(src + q);
                af[i][q] = t[0]; af[i][q + 1] = t[1]; af[i][q + 2] = t[2]; af[i][q + 3] = t[3];
            }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const float *src = Bs + (wn * TN + j * MF + MM::idx(lane)) * LDSW + MM::grp(lane) * KPL;
#pragma unroll
            for (int q = 0; q < KPL; q += 4) {
                const f32x4v t = *(const f32x4v *)(src + q);
                bf[j][q] = t[0]; bf[j][q + 1] = t[1]; bf[j][q + 2] = t[2]; bf[j][q + 3] = t[3];
            }
        }
#pragma unroll
        for (int s = 0; s < KPL; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = MM::mma(af[i][s], bf[j][s], acc[i][j]);
    }
    }

    // ------------------------------------------------------------------ epilogue
    int ncol[FN];
    float bcol[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        ncol[j] = n0 + wn * TN + j * MF + MM::col(lane);
        bcol[j] = ncol[j] < g.N ? epi.colv(ncol[j]) : 0.f;
    }
    const long wrow0 = m0 + wm * TM;
    // Row m = wrow0 + off (off < TM) is decomposed from the wave's first row, so only
    // small quotients (qdiv) are needed per row group.  With Mimg and OW multiples of 4
    // a group of four consecutive rows is four neighbouring pixels of one output row.
    const long imgw = DENSE ? wrow0 : ldiv64(wrow0, g.rMd);
    const int pw = (int)(wrow0 - imgw * Mimg);
    // every row of the wave's tile exists and belongs to img imgw (the usual case for
    // convolutions): the fast epilogue applies
    const bool uniform = wrow0 + TM <= M && pw + TM <= Mimg;
    const float rM = g.rM, rOW = g.rOW;
    const bool quad = (Mimg % 4 == 0) && (g.OW % 4 == 0);
    auto rowfn4 = [&](int i, int vg, int (&img)[4], int (&dp)[4]) -> bool {
        const int off = i * MF + MM::row(4 * vg, lane);
        if (DENSE) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                img[q] = wrow0 + off + q < M ? (int)(wrow0 + off + q) : -1;
                dp[q] = 0;
            }
            return false;
        }
        if (quad) {
            int p = pw + off;
            const int k = qdiv(p, rM);
            p -= k * (int)Mimg;
            const int oy = qdiv(p, rOW), ox = p - oy * g.OW;
            const int iv = imgw + k < n_img ? (int)(imgw + k) : -1;
            const int b = (oy * g.ostr + g.oy0) * g.DW + ox * g.ostr + g.ox0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                img[q] = iv;
                dp[q] = b + q * g.ostr;
            }
            return true;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int p = pw + off + q;
            const int k = qdiv(p, rM);
            p -= k * (int)Mimg;
            const int oy = qdiv(p, rOW), ox = p - oy * g.OW;
            img[q] = imgw + k < n_img ? (int)(imgw + k) : -1;
            dp[q] = (oy * g.ostr + g.oy0) * g.DW + ox * g.ostr + g.ox0;
        }
        return false;
    };
    const bool fast = !DENSE && uniform && quad && n0 + BN <= g.N;
    tile_epilogue<Epi, MF, FM, FN, !DENSE>(epi, acc, ncol, bcol, g.N, rowfn4, lane, fast,
                                           fast ? (int)imgw : -1);
}

// ---------------------------------------------------------------------- dispatch
template <class Epi, int MF, int BM, int BN, int WGM, int WGN, bool DMAG = false>
hipError_t launch_cfg(const GeomSet &gs, const float *A, long n_img, const Epi &epi,
                      hipStream_t st) {
    const Geom &g0 = gs.g[0];
    long Mmax = 0;
    for (int i = 0; i < gs.n; ++i) {
        const long M = n_img * (long)gs.g[i].OH * gs.g[i].OW;
        if (M > Mmax) Mmax = M;
    }
    if (Mmax == 0) return hipSuccess;
    const long tiles = ((Mmax + BM - 1) / BM) * ((g0.N + BN - 1) / BN) * gs.n;
    if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)tiles);   // tile order: xcd_tile
    const bool dense = g0.H == 1 && g0.W == 1 && g0.kh == 1 && g0.kw == 1;
    const bool vec = (g0.C % 4 == 0) && (g0.K % 4 == 0);
    for (int i = 0; i < gs.n; ++i) {
        if (!dense && gs.g[i].K > KDEC_MAX) return hipErrorInvalidValue;  // layer too wide
        if ((long)gs.g[i].OH * gs.g[i].OW > (1L << 20)) return hipErrorInvalidValue;  // qdiv range
    }
    bool k16 = true;
    for (int i = 0; i < gs.n; ++i) k16 = k16 && gs.g[i].K % BK == 0;
    if (DMAG && dense && vec && k16)
        hipLaunchKernelGGL((k_gemm<Epi, MF, BM, BN, WGM, WGN, true, true, DMAG>), grid, dim3(256), 0, st, gs, A, n_img, epi);
    else if (dense && vec)
        hipLaunchKernelGGL((k_gemm<Epi, MF, BM, BN, WGM, WGN, true, true>), grid, dim3(256), 0, st, gs, A, n_img, epi);
    else if (dense)
        hipLaunchKernelGGL((k_gemm<Epi, MF, BM, BN, WGM, WGN, true, false>), grid, dim3(256), 0, st, gs, A, n_img, epi);
    else if (vec)
        hipLaunchKernelGGL((k_gemm<Epi, MF, BM, BN, WGM, WGN, false, true>), grid, dim3(256), 0, st, gs, A, n_img, epi);
    else
        hipLaunchKernelGGL((k_gemm<Epi, MF, BM, BN, WGM, WGN, false, false>), grid, dim3(256), 0, st, gs, A, n_img, epi);
    return hipGetLastError();
}

// Tile configurations: {MFMA size, BM, BN, wave grid}.
//   0: 32x32 MFMA, 128x128, 2x2   1: 32, 128x64, 2x2    2: 32, 256x32, 4x1
//   3: 16x16 MFMA, 256x16, 4x1    4: 32, 256x64, 4x1    5: 32, 256x128, 4x1
//   6: 32, 128x32, 4x1 (one 32x32 tile per wave: fewest registers)
//   7: 16x16 MFMA, 128x32, 2x2    8: 32, 128x64, 4x1
//   9, 10: 8 and 1 with the k chunks by LDS DMA (dense products with K % 16 == 0)
constexpr int kGemmCfgs = 11;
const int kCfgBN[kGemmCfgs] = {128, 64, 32, 16, 64, 128, 32, 32, 64, 64, 64};

int default_cfg(int N) {
    if (N >= 128) return 0;
    if (N >= 64) return 1;
    if (N >= 32) return 2;
    return 3;
}

template <class Epi>
hipError_t dispatch(const GeomSet &gs, const float *A, long n_img, const Epi &epi, hipStream_t st,
                    int cfg) {
    if (cfg < 0 || cfg >= kGemmCfgs) cfg = default_cfg(gs.g[0].N);
    switch (cfg) {
    case 0: return launch_cfg<Epi, 32, 128, 128, 2, 2>(gs, A, n_img, epi, st);
    case 1: return launch_cfg<Epi, 32, 128, 64, 2, 2>(gs, A, n_img, epi, st);
    case 2: return launch_cfg<Epi, 32, 256, 32, 4, 1>(gs, A, n_img, epi, st);
    case 3: return launch_cfg<Epi, 16, 256, 16, 4, 1>(gs, A, n_img, epi, st);
    case 4: return launch_cfg<Epi, 32, 256, 64, 4, 1>(gs, A, n_img, epi, st);
    case 6: return launch_cfg<Epi, 32, 128, 32, 4, 1>(gs, A, n_img, epi, st);
    case 7: return launch_cfg<Epi, 16, 128, 32, 2, 2>(gs, A, n_img, epi, st);
    case 8: return launch_cfg<Epi, 32, 128, 64, 4, 1>(gs, A, n_img, epi, st);
    case 9: return launch_cfg<Epi, 32, 128, 64, 4, 1, true>(gs, A, n_img, epi, st);
    case 10: return launch_cfg<Epi, 32, 128, 64, 2, 2, true>(gs, A, n_img, epi, st);
    default: return launch_cfg<Epi, 32, 256, 128, 4, 1>(gs, A, n_img, epi, st);
    }
}

}  // namespace

int gemm_candidates(const GeomSet &gs, int *cfgs, int cap) {
    // a tile wider than the padded N only repeats zero columns
    const int N = gs.g[0].N;
    int n = 0;
    const Geom &g = gs.g[0];
    const bool dma = g.H == 1 && g.W == 1 && g.kh == 1 && g.kw == 1 && g.C % 4 == 0 &&
                     g.K % BK == 0;
    for (int c = 0; c < kGemmCfgs && n < cap; ++c) {
        if (c >= 9 && !dma) continue;
        if (kCfgBN[c] <= 16 * ((N + 15) / 16) || c == default_cfg(N)) cfgs[n++] = c;
    }
    return n;
}

hipError_t gemm_relax_cfg(const GeomSet &gs, const float *A, long n_img, const RelaxParams &p,
                          hipStream_t st, int cfg) {
    return dispatch(gs, A, n_img, dev::EpiRelax{p}, st, cfg);
}
hipError_t gemm_conc_cfg(const GeomSet &gs, const float *A, long n_img, const ConcParams &p,
                         hipStream_t st, int cfg) {
    return dispatch(gs, A, n_img, dev::EpiConc{p}, st, cfg);
}
hipError_t gemm_adj_cfg(const GeomSet &gs, const float *A, long n_img, const AdjParams &p,
                        hipStream_t st, int cfg) {
    return dispatch(gs, A, n_img, dev::EpiAdj{p}, st, cfg);
}
hipError_t gemm_fwd_cfg(const GeomSet &gs, const float *A, long n_img, const FwdParams &p,
                        hipStream_t st, int cfg) {
    return dispatch(gs, A, n_img, dev::EpiFwd{p}, st, cfg);
}

int plan_candidates(const GeomSet &gs, Plan *out, int cap) {
    int n = 0;
    int cc[kMaxCandidates], mode[kMaxCandidates];
    const int nd = direct_candidates(gs, cc, mode, kMaxCandidates);
    for (int i = 0; i < nd && n < cap; ++i) {
        out[n].path = 1;
        out[n].cfg = mode[i];
        out[n].cc = cc[i];
        ++n;
    }
    int cf[kMaxCandidates];
    const int ng = gemm_candidates(gs, cf, kMaxCandidates);
    for (int i = 0; i < ng && n < cap; ++i) {
        out[n].path = 2;
        out[n].cfg = cf[i];
        out[n].cc = 0;
        ++n;
    }
    return n;
}

#define BOUND_PRODUCT(NAME, PARAMS, DIRECT, CFG)                                             \
    hipError_t NAME(const GeomSet &gs, const float *A, long n_img, const PARAMS &p,          \
                    hipStream_t st, const Plan &plan) {                                      \
        if (plan.path != 2) {                                                                \
            bool used = false;                                                               \
            const hipError_t e = DIRECT(gs, A, n_img, p, st, plan.path == 1 ? plan.cc : 0,      \
                                        plan.cfg, &used);                                     \
            if (used || e != hipSuccess) return e;                                           \
        }                                                                                    \
        return CFG(gs, A, n_img, p, st, plan.path == 2 ? plan.cfg : -1);                     \
    }
BOUND_PRODUCT(gemm_relax, RelaxParams, direct_relax, gemm_relax_cfg)
BOUND_PRODUCT(gemm_conc, ConcParams, direct_conc, gemm_conc_cfg)
BOUND_PRODUCT(gemm_adj, AdjParams, direct_adj, gemm_adj_cfg)
BOUND_PRODUCT(gemm_fwd, FwdParams, direct_fwd, gemm_fwd_cfg)
#undef BOUND_PRODUCT

}  // namespace bp
