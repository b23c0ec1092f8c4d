// LDS-tiled direct convolution kernels for gfx950, used for the convolutional products
// of the bound pass and its adjoint when the layer geometry fits (otherwise the
// implicit-GEMM kernel in gemm.hip runs).
//
// A block owns 256 output pixels -- whole images when an image has <= 256 pixels,
// otherwise a band of full-width output rows -- and all BN output channels.  For each
// chunk of CC input channels it stages the input tile with its halo and the chunk's
// weights (all taps) in LDS once; every tap of the convolution then reads its operands
// from LDS, so each input element is fetched from L2/HBM once per block instead of once
// per tap.  v_mfma_f32_32x32x2f32 serves BN >= 32, v_mfma_f32_16x16x4f32 BN = 16.
// The same fused epilogues as the GEMM kernel apply (device_common.h).
//
// k_conv_valu covers products with at most 4 output channels (the first layer's
// transposed convolution back to a 3-channel input), where a 16-wide MFMA tile would
// waste most of its work: one thread per output pixel, plain FP32 FMAs of LDS inputs
// and scalar-loaded weights.
#include "device_common.h"

namespace bp {
namespace {

using namespace dev;

struct ConvTile {
    int G;         // images per block (whole-image tiles), else 1
    int TR;        // output rows per block
    int tiles_y;   // row bands per image
    int IH, IW;    // LDS input tile
    int CS;        // LDS channel stride (>= CC)
    int CC, lcc;   // channels per chunk (power of two) and its log2; CC = C when C < 4
    int nchunk;
    int T;         // taps kh * kw
    int KB;        // padded k per chunk (multiple of 16)
    int WS;        // LDS weight row stride
    int in_floats; // G * IH * IW * CS
    // fl(1 / d) of the divisors the kernels split indices by (qdiv), set on the host
    float rTY, rCC, rKW, rTP, rIH, rIW, rPin, rPw, rC4, rTK, rKB, rSPP, rSPR;
    // DMA staging: a thread's slots are tid, tid + 256, ...; these are the mixed-radix
    // digits of a 256-slot step of the input tile (channel quad, pixel column, row, image)
    // and of the weight tile (k quad, output row), each below its radix but the last
    int dC4, dIX, dIY, dGI, dK4, dN;
    int rowdma;    // DMA staging of the input tile by rows (else by 256-slot steps)
};

// Stage the input tile (channels [c0, c0+CC)) of images img0.. into LDS, zero outside.
template <bool VEC>
__device__ inline void stage_input(float *In, const ConvTile &ct, const Geom &g, const float *X,
                                   long img0, long n_img, int iy0, int ix0, int c0) {
    const int tid = threadIdx.x;
    if (VEC) {
        const int c4n = ct.CC >> 2;
        const int total = ct.G * ct.IH * ct.IW * c4n;
        for (int e = tid; e < total; e += 256) {
            const int pix = qdiv(e, ct.rC4), c4 = e - pix * c4n;
            const int t2 = qdiv(pix, ct.rIW), ix = pix - t2 * ct.IW;
            const int gi = qdiv(t2, ct.rIH), iy = t2 - gi * ct.IH;
            const long img = img0 + gi;
            const int y = iy0 + iy, x = ix0 + ix;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (img < n_img && (unsigned)y < (unsigned)g.H && (unsigned)x < (unsigned)g.W)
                v = *(const float4 *)(X + ((img * g.H + y) * (long)g.W + x) * g.C + c0 + 4 * c4);
            *(float4 *)(In + ((gi * ct.IH + iy) * ct.IW + ix) * ct.CS + 4 * c4) = v;
        }
    } else {  // C < 4: one chunk, channels padded with zeros up to CS = 4
        // The first SP pixels of every thread are loaded together before any LDS store
        // (one memory latency for the tile instead of one per pixel); larger tiles
        // continue one pixel at a time.
        constexpr int SP = 4;
        const int total = ct.G * ct.IH * ct.IW;
        auto src_of = [&](int e, int &dst) -> const float * {
            const int t2 = qdiv(e, ct.rIW), ix = e - t2 * ct.IW;
            const int gi = qdiv(t2, ct.rIH), iy = t2 - gi * ct.IH;
            const long img = img0 + gi;
            const int y = iy0 + iy, x = ix0 + ix;
            dst = ((gi * ct.IH + iy) * ct.IW + ix) * ct.CS;
            return img < n_img && (unsigned)y < (unsigned)g.H && (unsigned)x < (unsigned)g.W
                       ? X + ((img * g.H + y) * (long)g.W + x) * g.C
                       : nullptr;
        };
        float v[SP][4];
        int dst[SP];
#pragma unroll
        for (int i = 0; i < SP; ++i) {
            const int e = tid + i * 256;
            dst[i] = -1;
            v[i][0] = v[i][1] = v[i][2] = v[i][3] = 0.f;
            if (e < total) {
                const float *src = src_of(e, dst[i]);
                if (src) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        if (c < g.C) v[i][c] = src[c];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < SP; ++i)
            if (dst[i] >= 0) *(float4 *)(In + dst[i]) = make_float4(v[i][0], v[i][1], v[i][2], v[i][3]);
        for (int e = tid + SP * 256; e < total; e += 256) {
            int d;
            const float *src = src_of(e, d);
            float w[4] = {0.f, 0.f, 0.f, 0.f};
            if (src)
                for (int c = 0; c < g.C; ++c) w[c] = src[c];
            *(float4 *)(In + d) = make_float4(w[0], w[1], w[2], w[3]);
        }
    }
}

// Stage weights of output channels [n0, n0+BN) for channels [c0, c0+CC), all taps:
// Wl[n][t*CC + c] = Bt[n0+n][t*C + c0 + c]; zero for k >= T*CC (padding to KB).
// The first SW elements of every thread are loaded together before any LDS store.
__device__ inline void stage_weights(float *Wl, const ConvTile &ct, const Geom &g, int BN, int n0, int c0) {
    constexpr int SW = 4;
    const int total = BN * ct.KB;
    const int TC = ct.T * ct.CC;
    auto one = [&](int e, int &dst) -> float {
        const int n = qdiv(e, ct.rKB), k = e - n * ct.KB;
        dst = n * ct.WS + k;
        if (k >= TC) return 0.f;
        const int t = qdiv(k, ct.rCC), c = k - t * ct.CC;
        return g.Bt[(long)(n0 + n) * g.Kp + t * g.C + c0 + c];
    };
    float v[SW];
    int dst[SW];
#pragma unroll
    for (int i = 0; i < SW; ++i) {
        const int e = threadIdx.x + i * 256;
        dst[i] = -1;
        v[i] = e < total ? one(e, dst[i]) : 0.f;
    }
#pragma unroll
    for (int i = 0; i < SW; ++i)
        if (dst[i] >= 0) Wl[dst[i]] = v[i];
    for (int e = threadIdx.x + SW * 256; e < total; e += 256) {
        int d;
        const float w = one(e, d);
        Wl[d] = w;
    }
}

// Register prefetch capacity per thread (float4s) for the next chunk's input tile and
// weights; plan_chunk keeps every tile within it.
constexpr int MAX_IN4 = 8, MAX_W4 = 6;
// DMA staging: slots per thread (input, weights), one offset register each
constexpr int DMA_IN4 = 12, DMA_W4 = 6;
// ... and a smaller set for tiles that need no more (fewer set-up instructions)
constexpr int DMA_SMALL_IN4 = 8, DMA_SMALL_W4 = 4;
// input slots of the narrow-output VALU kernel's DMA staging, and its row segments when
// it stages by rows
constexpr int VALU_DMA_IN4 = 8, DMA_ROW_SEG = 4;

// Element walk over a [rows][P] float4 grid: thread tid visits e = tid, tid + 256, ...;
// the row / column of each visit advance incrementally (one division per thread).
struct Walk {
    int r, p, dr, dp, P;
    __device__ Walk(int P_, float rP) : P(P_) {
        r = qdiv(threadIdx.x, rP);
        p = threadIdx.x - r * P;
        dr = 256 / P;
        dp = 256 - dr * P;
    }
    __device__ void next() {
        p += dp;
        r += dr;
        if (p >= P) {
            p -= P;
            ++r;
        }
    }
};

template <class Epi, int MF, int BN, bool VEC, int NIN, int NW, bool DMA>
__global__ __launch_bounds__(256) void k_conv(const GeomSet gs, const ConvTile ct,
                                              const float *__restrict__ X, const long n_img,
                                              const Epi epi) {
    using MM = Mma<MF>;
    using acc_t = typename MM::acc_t;
    constexpr int FM = 64 / MF, FN = BN / MF, KPL = MM::KPL;
    extern __shared__ __attribute__((aligned(16))) float smem[];
    float *In = smem;
    float *Wl = smem + ct.in_floats;
    int *koff = (int *)(Wl + BN * ct.WS);     // [KB] A-operand offset of k inside the tile

    const TileIdx ti = xcd_tile(gs.g[0].N / BN, gs.n);
    const Geom &g = gs.g[ti.z];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long grp = ldiv_by(ti.x, ct.tiles_y, ct.rTY);
    const int band = (int)(ti.x - grp * ct.tiles_y);
    const long img0 = grp * ct.G;
    if (img0 >= n_img) return;
    const int oyb = band * ct.TR;
    const int n0 = ti.y * BN;
    const int tile_px = ct.TR * g.OW;
    const int iy0 = oyb * g.stride - g.pad_y, ix0 = -g.pad_x;
    const int TC = ct.T * ct.CC;

    // k -> offset of (tap, channel) inside the LDS input tile; padding k reads offset 0
    // against zero weights.
    for (int k = tid; k < ct.KB; k += 256) {
        int o = 0;
        if (k < TC) {
            const int t = qdiv(k, ct.rCC), c = k - t * ct.CC;
            const int ty = qdiv(t, ct.rKW), tx = t - ty * g.kw;
            o = (ty * ct.IW + tx) * ct.CS + c;
        }
        koff[k] = o;
    }

    // LDS offset of the top-left input of each A row this lane supplies.
    int abase[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int lr = wave * 64 + i * MF + MM::idx(lane);
        const int gi = qdiv(lr, ct.rTP), q = lr - gi * tile_px;
        const int py = qdiv(q, g.rOW), px = q - py * g.OW;
        abase[i] = ((gi * ct.IH + py * g.stride) * ct.IW + px * g.stride) * ct.CS;
    }
    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < MM::NACC; ++v) acc[i][j][v] = 0.f;

    // Staging of one channel chunk through registers (VEC: CC is a power of two >= 4).
    // The tile position of each staged float4 is the same for every chunk; only the
    // channel offset c0 changes, so global and LDS offsets are computed once here
    // (global offsets relative to the block's first image; -1 marks zero padding).
    //
    // DMA: the chunk goes from global memory straight into LDS (buffer loads with the
    // LDS destination, 16 bytes per lane at consecutive LDS addresses), so no staging
    // registers are held across the k-loop.  LDS float4 slot s = i * 256 + tid of the
    // input tile (pixel, channel quad; the rows are unpadded, which keeps the tile small
    // enough for one more block per CU) and of the weight tile (output, k quad incl.
    // padding) is fetched by that thread; slots that are always zero (spatial padding, k
    // past the chunk) are written once, padding columns never, and slots past the last
    // image of a partial group read out of range of the buffer (no access) and feed only
    // rows the epilogue drops.
    //
    // With ct.rowdma (LDS rows of 64 slots or more) the input tile goes by rows instead:
    // LDS row r = gi * IH + iy (the IW * spp slots of input row iy0 + iy of image gi) is
    // fetched as 64-slot segments, one DMA instruction each.  A lane's source offset
    // inside a row is then the same for every row, image and chunk and the row's offset
    // is wave-uniform, so the per-slot index arithmetic of the set-up goes away; the tile
    // is zeroed once, and rows of spatial padding or of images past the batch are never
    // fetched.
    const int c4s = VEC ? ct.lcc - 2 : 0;             // log2(CC / 4)
    const int Pin = ct.IW << c4s, Rin = ct.G * ct.IH;  // input grid [G*IH][IW*CC/4]
    const int Pw = ct.KB >> 2;                         // weight grid [BN][KB/4]
    const float *Xb = X + img0 * (long)g.H * g.W * g.C;
    const float *Bb = g.Bt + (long)n0 * g.Kp;
    int gin[NIN], lin[NIN], gw[NW], lw[NW];
    if (VEC && DMA && ct.rowdma) {
        // segment q of a row: slot q * 64 + lane -> pixel column ix, channel quad c4
        // (spp = CS / 4 slots per pixel, a power of two); -1: nothing to fetch
        const int lsp = ct.lcc - 2, rs = ct.IW << lsp;
#pragma unroll
        for (int q = 0; q < NIN / 4; ++q) {
            const int sl = q * 64 + lane;
            const int x = ix0 + (sl >> lsp), c4 = sl & ((1 << lsp) - 1);
            gin[q] = sl < rs && (unsigned)x < (unsigned)g.W ? (x * g.C + 4 * c4) * 4 : -1;
        }
        for (int e = tid; e < (ct.in_floats >> 2); e += 256)
            *(float4 *)(In + 4 * e) = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();   // the zeros land before any DMA write to the same slots
    } else if (VEC && DMA) {
        // slot sl = ((gi * IH + iy) * IW + ix) * spp + c4: the first slot is decomposed
        // with quotients, the later ones step its digits by 256 slots (host-computed)
        const int spp = ct.CS >> 2, S_in = ct.in_floats >> 2;
        int c4, ix, iy, gi;
        {
            const int pix = qdiv(tid, ct.rSPP);
            c4 = tid - pix * spp;
            const int row = qdiv(pix, ct.rIW);
            ix = pix - row * ct.IW;
            gi = qdiv(row, ct.rIH);
            iy = row - gi * ct.IH;
        }
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            const int sl = i * 256 + tid;
            int o = -2;
            if (sl < S_in) {
                o = -1;
                const int y = iy0 + iy, x = ix0 + ix;
                if (c4 < (ct.CC >> 2) && (unsigned)y < (unsigned)g.H && (unsigned)x < (unsigned)g.W)
                    o = (((gi * g.H + y) * g.W + x) * g.C + 4 * c4) * 4;
                else if (c4 == (ct.CC >> 2))
                    o = -2;                           // row padding (if any): never read
            }
            gin[i] = o;
            if (o == -1) *(float4 *)(In + 4 * sl) = make_float4(0.f, 0.f, 0.f, 0.f);
            c4 += ct.dC4;
            const int cc = c4 >= spp;
            c4 -= cc ? spp : 0;
            ix += ct.dIX + cc;
            const int cx = ix >= ct.IW;
            ix -= cx ? ct.IW : 0;
            iy += ct.dIY + cx;
            const int cy = iy >= ct.IH;
            iy -= cy ? ct.IH : 0;
            gi += ct.dGI + cy;
        }
    }
    if (VEC && DMA) {
        // weight slot sl = n * spr + k4: the first one decomposed with a quotient, the
        // later ones step its digits by 256 slots (host-computed); steps past the tile
        // (a wave-uniform test) are skipped
        const int spr = ct.WS >> 2, S_w = BN * spr;
        int n = qdiv(tid, ct.rSPR), k4 = tid - n * spr;
#pragma unroll
        for (int i = 0; i < NW; ++i) gw[i] = -2;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            if (i * 256 >= S_w) break;
            const int sl = i * 256 + tid;
            int o = -2;
            if (sl < S_w) {
                const int k = 4 * k4;
                if (k4 < (ct.KB >> 2))
                    o = k < TC ? (n * g.Kp + (k >> ct.lcc) * g.C + (k & (ct.CC - 1))) * 4 : -1;
            }
            gw[i] = o;
            if (o == -1) *(float4 *)(Wl + 4 * sl) = make_float4(0.f, 0.f, 0.f, 0.f);
            k4 += ct.dK4;
            const int ck = k4 >= spr;
            k4 -= ck ? spr : 0;
            n += ct.dN + ck;
        }
    } else if (VEC) {
        Walk w(Pin, ct.rPin);
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            gin[i] = -1;
            lin[i] = -1;
            if (w.r < Rin) {
                const int gi = qdiv(w.r, ct.rIH), iy = w.r - gi * ct.IH;
                const int ix = w.p >> c4s, c4 = w.p & ((1 << c4s) - 1);
                const int y = iy0 + iy, x = ix0 + ix;
                lin[i] = (w.r * ct.IW + ix) * ct.CS + 4 * c4;
                if (img0 + gi < n_img && (unsigned)y < (unsigned)g.H && (unsigned)x < (unsigned)g.W)
                    gin[i] = ((gi * g.H + y) * g.W + x) * g.C + 4 * c4;
            }
            w.next();
        }
        Walk ww(Pw, ct.rPw);
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            gw[i] = -1;
            lw[i] = -1;
            const int k = ww.p << 2;
            if (ww.r < BN) {
                lw[i] = ww.r * ct.WS + k;
                if (k < TC) gw[i] = ww.r * g.Kp + (k >> ct.lcc) * g.C + (k & (ct.CC - 1));
            }
            ww.next();
        }
    }
    float4 rin[DMA ? 1 : NIN], rw[DMA ? 1 : NW];
    auto load_chunk = [&](int c0) {
        if (DMA) return;
#pragma unroll
        for (int i = 0; i < NIN; ++i)
            rin[i] = gin[i] >= 0 ? *(const float4 *)(Xb + gin[i] + c0) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int i = 0; i < NW; ++i)
            rw[i] = gw[i] >= 0 ? *(const float4 *)(Bb + gw[i] + c0) : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto store_chunk = [&]() {
        if (DMA) return;
#pragma unroll
        for (int i = 0; i < NIN; ++i)
            if (lin[i] >= 0) *(float4 *)(In + lin[i]) = rin[i];
#pragma unroll
        for (int i = 0; i < NW; ++i)
            if (lw[i] >= 0) *(float4 *)(Wl + lw[i]) = rw[i];
    };
    // buffer extents: the block's image group (clipped to the images that exist) and
    // its weight rows
    const long nvg = n_img - img0 < ct.G ? n_img - img0 : ct.G;
    const int xbytes = (int)(nvg * g.H * g.W * g.C * 4), wbytes = BN * g.Kp * 4;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    auto dma_chunk = [&](int c0) {
        if (ct.rowdma) {
            // rows wv, wv + 4, ... of the tile, (gi, iy) stepped by 4 rows (wave-uniform)
            const int rs = ct.IW << (ct.lcc - 2), nrow = ct.G * ct.IH;
            int gi = 0, iy = wv;
            while (iy >= ct.IH) { iy -= ct.IH; ++gi; }
            for (int r = wv; r < nrow; r += 4) {
                const int y = iy0 + iy;
                if ((unsigned)y < (unsigned)g.H && img0 + gi < n_img) {
                    const int ro = (((gi * g.H + y) * g.W) * g.C + c0) * 4;
                    float *dst = In + r * rs * 4;
#pragma unroll
                    for (int q = 0; q < NIN / 4; ++q)
                        if (q * 64 < rs && gin[q] >= 0) lds_dma16(Xb, xbytes, dst + q * 256, gin[q] + ro);
                }
                iy += 4;
                while (iy >= ct.IH) { iy -= ct.IH; ++gi; }
            }
        } else {
#pragma unroll
            for (int i = 0; i < NIN; ++i)
                if (gin[i] >= 0) lds_dma16(Xb, xbytes, In + (i * 256 + wv * 64) * 4, gin[i] + 4 * c0);
        }
#pragma unroll
        for (int i = 0; i < NW; ++i)
            if (gw[i] >= 0) lds_dma16(Bb, wbytes, Wl + (i * 256 + wv * 64) * 4, gw[i] + 4 * c0);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    };

    const int kgrp = MM::grp(lane) * KPL;   // this lane's first k inside a 16-wide k block
    if (VEC && DMA) {
        dma_chunk(0);
    } else if (VEC) {
        load_chunk(0);
        store_chunk();
    } else {
        stage_input<false>(In, ct, g, X, img0, n_img, iy0, ix0, 0);
        stage_weights(Wl, ct, g, BN, n0, 0);
    }
    __syncthreads();
    for (int ch = 0; ch < ct.nchunk; ++ch) {
        const bool more = VEC && ch + 1 < ct.nchunk;
        if (more && !DMA) load_chunk((ch + 1) * ct.CC);      // in flight during this chunk's MFMAs
        for (int kb = 0; kb < ct.KB; kb += 16) {
            const int k = kb + kgrp;
            float af[FM][KPL], bf[FN][KPL];
            if (VEC) {   // KPL consecutive k share a tap: contiguous channels
                const int off = koff[k];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int q = 0; q < KPL; q += 4) {
                        const f32x4v a = *(const f32x4v *)(In + abase[i] + off + q);
                        af[i][q] = a[0]; af[i][q + 1] = a[1]; af[i][q + 2] = a[2]; af[i][q + 3] = a[3];
                    }
            } else {
#pragma unroll
                for (int q = 0; q < KPL; ++q) {
                    const int off = koff[k + q];
#pragma unroll
                    for (int i = 0; i < FM; ++i) af[i][q] = In[abase[i] + off];
                }
            }
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < KPL; q += 4) {
                    const f32x4v b = *(const f32x4v *)(Wl + (j * MF + MM::idx(lane)) * ct.WS + k + q);
                    bf[j][q] = b[0]; bf[j][q + 1] = b[1]; bf[j][q + 2] = b[2]; bf[j][q + 3] = b[3];
                }
#pragma unroll
            for (int s = 0; s < KPL; ++s)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = MM::mma(af[i][s], bf[j][s], acc[i][j]);
        }
        if (more) {
            __syncthreads();
            if (DMA)
                dma_chunk((ch + 1) * ct.CC);
            else
                store_chunk();
            __syncthreads();
        }
    }

    // ---------------------------------------------------------------- epilogue
    int ncol[FN];
    float bcol[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        ncol[j] = n0 + j * MF + MM::col(lane);
        bcol[j] = ncol[j] < g.N ? epi.colv(ncol[j]) : 0.f;
    }
    const float rTP = ct.rTP;
    const int gfirst = qdiv(wave * 64, rTP), glast = qdiv(wave * 64 + 63, rTP);
    const bool uniform = gfirst == glast && img0 + gfirst < n_img;
    // Local row lr < 256 -> (image of the block, pixel); with OW a multiple of 4 a group
    // of four consecutive rows is four neighbouring pixels of one output row.
    const float rOW = g.rOW;
    const bool quad = g.OW % 4 == 0;
    auto rowfn4 = [&](int i, int vg, int (&img)[4], int (&dp)[4]) -> bool {
        const int lr0 = wave * 64 + i * MF + MM::row(4 * vg, lane);
#pragma unroll
        for (int q = 0; q < (quad ? 1 : 4); ++q) {
            const int lr = lr0 + q;
            const int gi = qdiv(lr, rTP), r = lr - gi * tile_px;
            const int py = qdiv(r, rOW), px = r - py * g.OW;
            img[q] = img0 + gi < n_img ? (int)(img0 + gi) : -1;
            dp[q] = ((oyb + py) * g.ostr + g.oy0) * g.DW + (px * g.ostr + g.ox0);
        }
        if (quad) {
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                img[q] = img[0];
                dp[q] = dp[0] + q * g.ostr;
            }
        }
        return quad;
    };
    tile_epilogue<Epi, MF, FM, FN, true>(epi, acc, ncol, bcol, g.N, rowfn4, lane, uniform && quad,
                                         (int)(img0 + gfirst));
}

// One thread per output pixel, up to NMAX output channels, VALU FMAs from LDS.
// Input tile of all C channels (CC = C, C % 4 == 0) by LDS DMA in one pass: slot
// s = i * 256 + tid as in k_conv; spatial padding is written as zeros, a row padding
// column (when the rows are padded) not at all; images past the batch read nothing
// (their pixels are dropped).
template <int NIN>
__device__ inline void dma_input_tile(float *In, const ConvTile &ct, const Geom &g, const float *Xb,
                                      int xbytes, int iy0, int ix0) {
    const int tid = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int spp = ct.CS >> 2, S_in = ct.in_floats >> 2, c4n = ct.CC >> 2;
    if (ct.rowdma) {
        // by rows, as in k_conv (spp a power of two, rows of 64 .. 64 * DMA_ROW_SEG slots):
        // the tile is zeroed, then each wave fetches rows wv, wv + 4, ... segment by
        // segment; images past the batch read out of the buffer's range (their rows are
        // dropped)
        for (int e = tid; e < S_in; e += 256) *(float4 *)(In + 4 * e) = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        const int lsp = __builtin_ctz(spp), rs = ct.IW << lsp, nrow = ct.G * ct.IH;
        int so[DMA_ROW_SEG];
#pragma unroll
        for (int q = 0; q < DMA_ROW_SEG; ++q) {
            const int sl = q * 64 + (tid & 63);
            const int x = ix0 + (sl >> lsp), c4 = sl & (spp - 1);
            so[q] = sl < rs && c4 < c4n && (unsigned)x < (unsigned)g.W ? (x * g.C + 4 * c4) * 4 : -1;
        }
        int gi = 0, iy = wv;
        while (iy >= ct.IH) { iy -= ct.IH; ++gi; }
        for (int r = wv; r < nrow; r += 4) {
            const int y = iy0 + iy;
            if ((unsigned)y < (unsigned)g.H) {
                const int ro = ((gi * g.H + y) * g.W) * g.C * 4;
                float *dst = In + r * rs * 4;
#pragma unroll
                for (int q = 0; q < DMA_ROW_SEG; ++q)
                    if (q * 64 < rs && so[q] >= 0) lds_dma16(Xb, xbytes, dst + q * 256, so[q] + ro);
            }
            iy += 4;
            while (iy >= ct.IH) { iy -= ct.IH; ++gi; }
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        return;
    }
    // slot digits stepped by 256 slots as in k_conv's DMA staging
    int c4, ix, iy, gi;
    {
        const int pix = qdiv(tid, ct.rSPP);
        c4 = tid - pix * spp;
        const int row = qdiv(pix, ct.rIW);
        ix = pix - row * ct.IW;
        gi = qdiv(row, ct.rIH);
        iy = row - gi * ct.IH;
    }
#pragma unroll
    for (int i = 0; i < NIN; ++i) {
        const int sl = i * 256 + tid;
        if (sl < S_in) {
            const int y = iy0 + iy, x = ix0 + ix;
            if (c4 < c4n) {
                if ((unsigned)y < (unsigned)g.H && (unsigned)x < (unsigned)g.W)
                    lds_dma16(Xb, xbytes, In + (i * 256 + wv * 64) * 4,
                              (((gi * g.H + y) * g.W + x) * g.C + 4 * c4) * 4);
                else
                    *(float4 *)(In + 4 * sl) = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        c4 += ct.dC4;
        const int cc = c4 >= spp;
        c4 -= cc ? spp : 0;
        ix += ct.dIX + cc;
        const int cx = ix >= ct.IW;
        ix -= cx ? ct.IW : 0;
        iy += ct.dIY + cx;
        const int cy = iy >= ct.IH;
        iy -= cy ? ct.IH : 0;
        gi += ct.dGI + cy;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

template <class Epi, int NMAX, bool DMA>
__global__ __launch_bounds__(256) void k_conv_valu(const GeomSet gs, const ConvTile ct,
                                                   const float *__restrict__ X, const long n_img,
                                                   const Epi epi) {
    // The weights are read at block-uniform addresses through the constant address
    // space, so they arrive by scalar loads into SGPRs and feed the FMAs directly; only
    // the input tile goes through LDS.
    using cfloat = const __attribute__((address_space(4))) float;
    extern __shared__ __attribute__((aligned(16))) float smem[];
    float *In = smem;
    const TileIdx ti = xcd_tile(1, gs.n);
    const Geom &g = gs.g[ti.z];
    const int tid = threadIdx.x;
    const long grp = ldiv_by(ti.x, ct.tiles_y, ct.rTY);
    const int band = (int)(ti.x - grp * ct.tiles_y);
    const long img0 = grp * ct.G;
    if (img0 >= n_img) return;
    const int oyb = band * ct.TR;
    const int tile_px = ct.TR * g.OW;
    if (DMA) {
        const long nvg = n_img - img0 < ct.G ? n_img - img0 : ct.G;
        dma_input_tile<VALU_DMA_IN4>(In, ct, g, X + img0 * (long)g.H * g.W * g.C,
                                     (int)(nvg * g.H * g.W * g.C * 4), oyb * g.stride - g.pad_y,
                                     -g.pad_x);
    } else {
        stage_input<true>(In, ct, g, X, img0, n_img, oyb * g.stride - g.pad_y, -g.pad_x, 0);
    }
    __syncthreads();
    const int gi = qdiv(tid, ct.rTP), q = tid - gi * tile_px;
    const int py = qdiv(q, g.rOW), px = q - py * g.OW;
    const int base = ((gi * ct.IH + py * g.stride) * ct.IW + px * g.stride) * ct.CS;
    cfloat *Wg = (cfloat *)g.Bt;
    const int C = g.C, Kp = g.Kp, N = g.N;
    // weight row of output n (rows past N repeat the last one; their sums are unused)
    long wrow[NMAX];
#pragma unroll
    for (int n = 0; n < NMAX; ++n) wrow[n] = (long)(n < N ? n : N - 1) * Kp;
    float acc[NMAX];
#pragma unroll
    for (int n = 0; n < NMAX; ++n) acc[n] = 0.f;
    for (int ty = 0, t = 0; ty < g.kh; ++ty)
    for (int tx = 0; tx < g.kw; ++tx, ++t) {
        const float *a = In + base + (ty * ct.IW + tx) * ct.CS;
        cfloat *w = Wg + t * C;
        int c = 0;
        for (; c + 16 <= C; c += 16) {     // 16 channels: the weights in one batch of loads
            float wv[NMAX][16];
#pragma unroll
            for (int n = 0; n < NMAX; ++n)
#pragma unroll
                for (int u = 0; u < 16; ++u) wv[n][u] = w[wrow[n] + c + u];
            float4 av[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = *(const float4 *)(a + c + 4 * u);
#pragma unroll
            for (int n = 0; n < NMAX; ++n)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc[n] = fmaf(av[u].x, wv[n][4 * u], acc[n]);
                    acc[n] = fmaf(av[u].y, wv[n][4 * u + 1], acc[n]);
                    acc[n] = fmaf(av[u].z, wv[n][4 * u + 2], acc[n]);
                    acc[n] = fmaf(av[u].w, wv[n][4 * u + 3], acc[n]);
                }
        }
        for (; c < C; c += 4) {
            const float4 av = *(const float4 *)(a + c);
#pragma unroll
            for (int n = 0; n < NMAX; ++n) {
                cfloat *wn = w + wrow[n] + c;
                acc[n] = fmaf(av.x, wn[0], acc[n]);
                acc[n] = fmaf(av.y, wn[1], acc[n]);
                acc[n] = fmaf(av.z, wn[2], acc[n]);
                acc[n] = fmaf(av.w, wn[3], acc[n]);
            }
        }
    }
    const long img = img0 + gi;
    float r0 = 0.f, r1 = 0.f;
    const int dpix = ((oyb + py) * g.ostr + g.oy0) * g.DW + (px * g.ostr + g.ox0);
    if (img < n_img) {
        const auto rc = epi.row((int)img);
        typename Epi::Pre pre[NMAX];
#pragma unroll
        for (int n = 0; n < NMAX; ++n)
            if (n < g.N) {
                pre[n] = epi.pre(rc, dpix * g.N + n);
                epi.pre2(rc, pre[n]);
            }
#pragma unroll
        for (int n = 0; n < NMAX; ++n)
            if (n < g.N) epi.post(pre[n], rc, dpix, n, dpix * g.N + n, epi.colv(n), acc[n], r0, r1);
    }
    if (Epi::NRED > 0) {
        // a wave's 64 pixels lie in one image whenever an image has >= 64 pixels
        const int lane = tid & 63;
        const int wave = tid >> 6;
        const int gf = qdiv(wave * 64, ct.rTP), gl = qdiv(wave * 64 + 63, ct.rTP);
        if (gf == gl) {
            if (img0 + gf < n_img) reduce_wave(epi, r0, r1, img0 + gf, dpix, 0, lane);
        } else {
            if (img < n_img) put_row_sums(epi, img, dpix, 0, r0, r1);
        }
    }
}

// ---------------------------------------------------------------------- planning
constexpr int LDS_BUDGET = 80 * 1024;

// Tile the 256-pixel block over the output grid; false if the grid does not divide.
bool plan_tile(const Geom &g, ConvTile &ct) {
    const int px = g.OH * g.OW;
    if (px <= 256) {
        if (256 % px != 0) return false;
        ct.G = 256 / px;
        ct.TR = g.OH;
        ct.tiles_y = 1;
    } else {
        if (256 % g.OW != 0) return false;
        const int tr = 256 / g.OW;
        if (g.OH % tr != 0) return false;
        ct.G = 1;
        ct.TR = tr;
        ct.tiles_y = g.OH / tr;
    }
    ct.IH = (ct.TR - 1) * g.stride + g.kh;
    ct.IW = (g.OW - 1) * g.stride + g.kw;
    ct.T = g.kh * g.kw;
    return true;
}

float recip(int d) { return 1.0f / (float)(d > 0 ? d : 1); }

// Reciprocals of the tile's divisors for qdiv (after plan_tile / plan_chunk).
void set_tile_recips(const Geom &g, ConvTile &ct) {
    ct.rTY = recip(ct.tiles_y);
    ct.rCC = recip(ct.CC);
    ct.rKW = recip(g.kw);
    ct.rTP = recip(ct.TR * g.OW);
    ct.rIH = recip(ct.IH);
    ct.rIW = recip(ct.IW);
    ct.rPin = recip(ct.CC >= 4 ? ct.IW * (ct.CC >> 2) : ct.IW);
    ct.rPw = recip(ct.KB >> 2);
    ct.rC4 = recip(ct.CC >> 2);
    ct.rTK = recip(ct.T * g.C);
    ct.rKB = recip(ct.KB);
    ct.rSPP = recip(ct.CS >> 2);
    ct.rSPR = recip(ct.WS >> 2);
    const int spp = ct.CS >= 4 ? ct.CS >> 2 : 1, dp = 256 / spp, spr = ct.WS >> 2;
    const int drow = dp / (ct.IW > 0 ? ct.IW : 1), ih = ct.IH > 0 ? ct.IH : 1;
    ct.dC4 = 256 - dp * spp;
    ct.dIX = dp - drow * ct.IW;
    ct.dIY = drow % ih;
    ct.dGI = drow / ih;
    ct.dK4 = spr > 0 ? 256 % spr : 0;
    ct.dN = spr > 0 ? 256 / spr : 0;
}

bool same_shape(const GeomSet &gs) {
    for (int i = 1; i < gs.n; ++i)
        if (gs.g[i].OH != gs.g[0].OH || gs.g[i].OW != gs.g[0].OW || gs.g[i].kh != gs.g[0].kh ||
            gs.g[i].kw != gs.g[0].kw || gs.g[i].N != gs.g[0].N || gs.g[i].C != gs.g[0].C)
            return false;
    return true;
}

// Choose the channel chunk for the MFMA kernel (want = 0: the largest that fits, else
// exactly want); returns LDS bytes or 0 if nothing fits.
size_t plan_chunk(const Geom &g, int BN, int KPL, ConvTile &ct, int want = 0, bool dma = false) {
    if (g.C < 4) {
        ct.CC = g.C;
        ct.lcc = 0;
        ct.CS = 4;
        ct.nchunk = 1;
    } else {
        int best = 0;
        for (int cc = 64; cc >= KPL; cc >>= 1) {
            if (g.C % cc || (want && cc != want)) continue;
            const int cs = dma ? cc : cc + 4;   // DMA tiles unpadded (more blocks per CU)
            const size_t in = (size_t)ct.G * ct.IH * ct.IW * cs;
            const int kb = ((ct.T * cc + 15) / 16) * 16;
            const size_t w = (size_t)BN * (dma ? kb : kb + 4);
            const bool regs =
                dma ? in / 4 <= 256 * DMA_IN4 && w / 4 <= 256 * DMA_W4 &&
                          (size_t)ct.G * g.H * g.W * g.C * 4 < 0x7fffffffUL
                    : (size_t)ct.G * ct.IH * ct.IW * (cc / 4) <= 256 * MAX_IN4 &&
                          (size_t)BN * (kb / 4) <= 256 * MAX_W4;
            if (regs && (in + w + kb) * 4 <= LDS_BUDGET) { best = cc; break; }
        }
        if (!best) return 0;
        ct.CC = best;
        ct.lcc = __builtin_ctz(best);
        ct.CS = dma ? best : best + 4;
        ct.nchunk = g.C / best;
    }
    ct.KB = ((ct.T * ct.CC + 15) / 16) * 16;
    // weight rows padded by 4 floats against LDS bank conflicts of the B reads; DMA
    // tiles unpadded, which keeps their LDS footprint (and so the blocks per CU) down
    ct.WS = dma ? ct.KB : ct.KB + 4;
    ct.in_floats = ct.G * ct.IH * ct.IW * ct.CS;
    const size_t bytes = ((size_t)ct.in_floats + (size_t)BN * ct.WS + ct.KB) * 4;
    return bytes <= LDS_BUDGET ? bytes : 0;
}

// Allow the kernel the dynamic LDS it is planned with (above the default limit).
template <class K> hipError_t allow_lds(K kern) {
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               LDS_BUDGET);
}

// Register prefetch slots of a launch: a small set when the tile needs no more, which
// keeps the kernel's register count (and so its occupancy) down.
constexpr int SMALL_IN4 = 5, SMALL_W4 = 2;

template <class Epi, int MF, int BN, int NIN, int NW>
hipError_t launch_slots(const GeomSet &gs, const ConvTile &ct, size_t lds, const float *X,
                        long n_img, const Epi &epi, hipStream_t st, dim3 grid) {
    if (gs.g[0].C % 4 == 0) {
        static const hipError_t ok = allow_lds(k_conv<Epi, MF, BN, true, NIN, NW, false>);
        if (ok != hipSuccess) return ok;
        hipLaunchKernelGGL((k_conv<Epi, MF, BN, true, NIN, NW, false>), grid, dim3(256), lds, st, gs, ct, X, n_img, epi);
    } else {
        static const hipError_t ok = allow_lds(k_conv<Epi, MF, BN, false, NIN, NW, false>);
        if (ok != hipSuccess) return ok;
        hipLaunchKernelGGL((k_conv<Epi, MF, BN, false, NIN, NW, false>), grid, dim3(256), lds, st, gs, ct, X, n_img, epi);
    }
    return hipGetLastError();
}

template <class Epi, int MF, int BN>
hipError_t launch_mfma(const GeomSet &gs, const ConvTile &ct, size_t lds, const float *X, long n_img,
                       const Epi &epi, hipStream_t st, bool dma) {
    const long groups = (n_img + ct.G - 1) / ct.G;
    const dim3 grid((unsigned)(groups * ct.tiles_y * (gs.g[0].N / BN) * gs.n));   // xcd_tile order
    if (dma) {   // planned only with C % 4 == 0
        const bool dsmall = ct.in_floats / 4 <= 256 * DMA_SMALL_IN4 &&
                            BN * ct.WS / 4 <= 256 * DMA_SMALL_W4;
        // staging by rows where a row fills at least one 64-slot segment (narrower rows
        // would leave most lanes of each DMA instruction idle) and fits the offset
        // registers (NIN / 4 segments)
        ConvTile c2 = ct;
        const int rs = ct.IW * (ct.CS / 4);
        c2.rowdma = rs >= 64 && rs <= 64 * ((dsmall ? DMA_SMALL_IN4 : DMA_IN4) / 4);
        if (dsmall) {
            static const hipError_t ok =
                allow_lds(k_conv<Epi, MF, BN, true, DMA_SMALL_IN4, DMA_SMALL_W4, true>);
            if (ok != hipSuccess) return ok;
            hipLaunchKernelGGL((k_conv<Epi, MF, BN, true, DMA_SMALL_IN4, DMA_SMALL_W4, true>), grid,
                               dim3(256), lds, st, gs, c2, X, n_img, epi);
        } else {
            static const hipError_t ok = allow_lds(k_conv<Epi, MF, BN, true, DMA_IN4, DMA_W4, true>);
            if (ok != hipSuccess) return ok;
            hipLaunchKernelGGL((k_conv<Epi, MF, BN, true, DMA_IN4, DMA_W4, true>), grid, dim3(256),
                               lds, st, gs, c2, X, n_img, epi);
        }
        return hipGetLastError();
    }
    const bool small = gs.g[0].C % 4 == 0 &&
                       (size_t)ct.G * ct.IH * ct.IW * (ct.CC / 4) <= 256 * SMALL_IN4 &&
                       (size_t)BN * (ct.KB / 4) <= 256 * SMALL_W4;
    if (small) return launch_slots<Epi, MF, BN, SMALL_IN4, SMALL_W4>(gs, ct, lds, X, n_img, epi, st, grid);
    return launch_slots<Epi, MF, BN, MAX_IN4, MAX_W4>(gs, ct, lds, X, n_img, epi, st, grid);
}

int bn_for(int N) {
    if (N == 16) return 16;
    if (N == 32) return 32;
    if (N % 64 == 0) return 64;
    return 0;
}

template <class Epi>
hipError_t try_direct(const GeomSet &gs, const float *X, long n_img, const Epi &epi, hipStream_t st,
                      int want_cc, int mode, bool *used) {
    *used = false;
    const Geom &g = gs.g[0];
    if (g.H == 1 && g.W == 1 && g.kh == 1 && g.kw == 1) return hipSuccess;  // dense: GEMM
    if (!same_shape(gs) || n_img <= 0) return hipSuccess;
    ConvTile ct{};
    if (!plan_tile(g, ct)) return hipSuccess;
    const long groups = (n_img + ct.G - 1) / ct.G;
    if (groups * ct.tiles_y * (g.N / 4 + 1) * gs.n > 0x7fffffffL) return hipSuccess;
    if (g.N <= 4 && g.C % 4 == 0) {      // narrow output: VALU kernel
        ct.CC = g.C;
        ct.CS = mode == 3 ? g.C : g.C + 4;   // mode 3: DMA into unpadded rows
        ct.in_floats = ct.G * ct.IH * ct.IW * ct.CS;
        const size_t lds = (size_t)ct.in_floats * 4;
        if (lds > LDS_BUDGET) return hipSuccess;
        set_tile_recips(g, ct);
        const dim3 grid((unsigned)(groups * ct.tiles_y * gs.n));   // xcd_tile order
        // DMA staging when asked for and the tile fits its slots (int offsets inside a group)
        const bool dma = (mode == 1 || mode == 3) && ct.in_floats / 4 <= 256 * VALU_DMA_IN4 &&
                         (size_t)ct.G * g.H * g.W * g.C * 4 < 0x7fffffffUL;
        // by rows where the slots per pixel are a power of two and a row fills 64 .. 256
        // slots
        const int spp = ct.CS / 4, rs = ct.IW * spp;
        ct.rowdma = dma && (spp & (spp - 1)) == 0 && rs >= 64 && rs <= 64 * DMA_ROW_SEG;
        if (g.N == 3 && dma) {   // RGB input layers: no idle fourth output
            static const hipError_t ok = allow_lds(k_conv_valu<Epi, 3, true>);
            if (ok != hipSuccess) return ok;
            hipLaunchKernelGGL((k_conv_valu<Epi, 3, true>), grid, dim3(256), lds, st, gs, ct, X, n_img, epi);
        } else if (g.N == 3) {
            static const hipError_t ok = allow_lds(k_conv_valu<Epi, 3, false>);
            if (ok != hipSuccess) return ok;
            hipLaunchKernelGGL((k_conv_valu<Epi, 3, false>), grid, dim3(256), lds, st, gs, ct, X, n_img, epi);
        } else if (dma) {
            static const hipError_t ok = allow_lds(k_conv_valu<Epi, 4, true>);
            if (ok != hipSuccess) return ok;
            hipLaunchKernelGGL((k_conv_valu<Epi, 4, true>), grid, dim3(256), lds, st, gs, ct, X, n_img, epi);
        } else {
            static const hipError_t ok = allow_lds(k_conv_valu<Epi, 4, false>);
            if (ok != hipSuccess) return ok;
            hipLaunchKernelGGL((k_conv_valu<Epi, 4, false>), grid, dim3(256), lds, st, gs, ct, X, n_img, epi);
        }
        *used = true;
        return hipGetLastError();
    }
    const int BN = bn_for(g.N);
    if (!BN) return hipSuccess;
    // mode: bit 0 (1, 3) LDS DMA staging, bit 1 (2, 3) 16x16 MFMA tiles for 32 outputs
    const bool mf16 = BN == 32 && (mode == 2 || mode == 3);
    const int KPL = BN == 16 || mf16 ? Mma<16>::KPL : Mma<32>::KPL;
    const bool dma = (mode == 1 || mode == 3) && g.C % 4 == 0;
    const size_t lds = plan_chunk(g, BN, KPL, ct, want_cc, dma);
    if (!lds) return hipSuccess;
    set_tile_recips(g, ct);
    *used = true;
    if (BN == 16) return launch_mfma<Epi, 16, 16>(gs, ct, lds, X, n_img, epi, st, dma);
    if (BN == 32 && mf16) return launch_mfma<Epi, 16, 32>(gs, ct, lds, X, n_img, epi, st, dma);
    if (BN == 32) return launch_mfma<Epi, 32, 32>(gs, ct, lds, X, n_img, epi, st, dma);
    return launch_mfma<Epi, 32, 64>(gs, ct, lds, X, n_img, epi, st, dma);
}

}  // namespace

hipError_t direct_relax(const GeomSet &gs, const float *A, long n_img, const RelaxParams &p,
                        hipStream_t st, int cc, int mode, bool *used) {
    return try_direct(gs, A, n_img, EpiRelax{p}, st, cc, mode, used);
}
hipError_t direct_conc(const GeomSet &gs, const float *A, long n_img, const ConcParams &p,
                        hipStream_t st, int cc, int mode, bool *used) {
    return try_direct(gs, A, n_img, EpiConc{p}, st, cc, mode, used);
}
hipError_t direct_adj(const GeomSet &gs, const float *A, long n_img, const AdjParams &p,
                        hipStream_t st, int cc, int mode, bool *used) {
    return try_direct(gs, A, n_img, EpiAdj{p}, st, cc, mode, used);
}

hipError_t direct_fwd(const GeomSet &gs, const float *A, long n_img, const FwdParams &p,
                        hipStream_t st, int cc, int mode, bool *used) {
    return try_direct(gs, A, n_img, EpiFwd{p}, st, cc, mode, used);
}

int direct_candidates(const GeomSet &gs, int *cc, int *mode, int cap) {
    const Geom &g = gs.g[0];
    if (g.H == 1 && g.W == 1 && g.kh == 1 && g.kw == 1) return 0;
    if (!same_shape(gs)) return 0;
    ConvTile ct{};
    if (!plan_tile(g, ct)) return 0;
    if (g.N <= 4) {
        if (g.C % 4 != 0) return 0;
        int n = 0;
        for (int m = -1; m <= 3 && n < cap; m += 2) {   // registers, DMA, DMA unpadded
            cc[n] = 0;
            mode[n++] = m;
        }
        return n;
    }
    const int BN = bn_for(g.N);
    if (!BN) return 0;
    const int KPL = BN == 16 ? Mma<16>::KPL : Mma<32>::KPL;
    if (g.C < 4) {
        if (!plan_chunk(g, BN, KPL, ct)) return 0;
        cc[0] = 0;
        mode[0] = -1;
        return cap > 0 ? 1 : 0;
    }
    // each channel chunk with register staging (mode -1) and with LDS DMA staging (1);
    // 32-output products also with 16x16 MFMA tiles (modes 2, 3), which allow chunks of
    // 4 channels
    int n = 0;
    const int modes[4] = {-1, 1, 2, 3};
    for (int c = 64; c >= 4; c >>= 1) {
        for (int mi = 0; mi < (BN == 32 ? 4 : 2) && n < cap; ++mi) {
            const int m = modes[mi];
            const int kpl = m >= 2 ? Mma<16>::KPL : KPL;
            ConvTile t = ct;
            if (c >= kpl && g.C % c == 0 && plan_chunk(g, BN, kpl, t, c, m == 1 || m == 3)) {
                cc[n] = c;
                mode[n] = m;
                ++n;
            }
        }
    }
    return n;
}

}  // namespace bp
