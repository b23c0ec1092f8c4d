// Internal declarations shared by the gfx950 kernels and the host side of the library.
//
// Layout inside the library: every coefficient tensor is [img][H][W][C] (channels last),
// where img enumerates (instance, spec row) pairs; Linear layers are the 1x1 case.
// Neuron index j inside a layer is therefore (y * W + x) * C + c ("internal order");
// the C ABI uses the C-major order c * H * W + y * W + x.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bp {

// Implicit-GEMM geometry.  Row m of the GEMM is (img, oy, ox) over an OH x OW grid; the
// A operand gathers A[img][y][x][c] at y = oy*stride - pad_y + ky, x = ox*stride - pad_x
// + kx for k = (ky*kw + kx)*C + c (zero outside the source); B is packed as Bt[N][Kp];
// the result element (m, n) goes to destination pixel (oy*ostr + oy0, ox*ostr + ox0)
// of a [img][DH][DW][N] tensor.
struct Geom {
    int H, W, C;
    int OH, OW;
    int kh, kw, stride, pad_y, pad_x;
    int K, N, Kp;
    int DH, DW, ostr, oy0, ox0;
    float rOW, rM;             // fl(1 / OW), fl(1 / (OH * OW)) for the quotients of qdiv
    float rC, rKW;             // fl(1 / C), fl(1 / kw)
    double rMd;                // 1 / (OH * OW) in FP64 for row indices beyond 2^21
    const float *Bt;
};

// Reciprocals of a geometry's divisors, taken once on the host (the same correctly
// rounded FP32 quotients a kernel would form).
inline void set_recips(Geom &g) {
    const int m = g.OH * g.OW > 0 ? g.OH * g.OW : 1;
    g.rOW = 1.0f / (float)(g.OW > 0 ? g.OW : 1);
    g.rM = 1.0f / (float)m;
    g.rC = 1.0f / (float)(g.C > 0 ? g.C : 1);
    g.rKW = 1.0f / (float)(g.kw > 0 ? g.kw : 1);
    g.rMd = 1.0 / (double)m;
}

struct GeomSet {
    Geom g[4];
    int n;
};

// Per-neuron relaxation record (Lemma 1) for one instance:
// x = lower slope, y = upper slope, z = upper intercept; w = 0 for a stable neuron,
// -(q + 1) for a split neuron whose first entry in the instance's split list is q, and
// k + 1 for an unstable one, k its slot in the compact rows of saved coefficients (alpha
// free).  Records with w <= 0 have x = y and z = +-0: a split record carries the sign of
// its first entry's constraint in the sign bit of z (-0 for sign -1), which the adjoint
// needs for that entry's beta-gradient (the slope cannot tell it when l = u = 0).
typedef float4 Relax;

// ----- epilogue parameter blocks -----------------------------------------------------
// Deterministic row sums: each tile's partial sums of a row go to their own slot
// part[(img * nslot + dp * ncu + n0 / 16) * 2 + {0, 1}] (dp the destination pixel of the
// tile's first row, n0 its first column, ncu = ceil(N / 16)) of a zeroed workspace, and
// launch_det_reduce adds the slots to the accumulators in slot order.
struct DetSums {
    float *part;
    long nslot;
    int ncu;
};

struct RelaxParams {       // G_m = Lambda_m W_m  ->  Lambda_{m-1} = relax(G_m)
    float *out;            // Lambda_{m-1}  [img][D]
    float *save;           // G_m kept for the gradient (nullable): per img, the unstable
                           // neurons only, at slot w - 1 of their record
    const Relax *tab;      // relaxation table of layer m-1, row stride tab_ld
    long tab_ld;
    const float *bias;     // b_{m-1} per channel
    int chan;              // channels of layer m-1 (bias index = j % chan)
    long D;                // width of layer m-1
    float *s, *mag;        // per-img offset accumulator and |term| accumulator
    long img0;             // global img index of local img 0
    int rpi;               // imgs per instance
    float rrpi;            // fl(1 / rpi)
    const float *bsum;     // [nnz][rpi] split-multiplier term per first split entry and
                           // row, subtracted at the split neuron (nullable: no beta)
    DetSums det;           // deterministic row sums (det.part null: float atomics)
};

struct ConcParams {        // G_1 = Lambda_1 W_1  ->  concretise over the box
    const float *cen, *rad;  // [n_inst][d0] internal order
    long D;                // d0
    float *low, *mag;      // per-img accumulators
    float *save;           // G_1 kept (nullable)
    float *emit;           // coefficient output in C-major order (nullable)
    int chan, hw;          // input shape for the C-major index
    long img0;
    int rpi;
    float rrpi;
    DetSums det;
};

struct AdjParams {         // Lambda_bar_m = G_bar_m W_m^T + s_bar b_m  -> G_bar_{m+1}
    const float *sbar;     // per img: gradient of the offset (0 for infeasible instances)
    const float *bias;     // b_m per channel
    int chan;
    long D;                // width of layer m
    const float *gsave;    // saved G_{m+1} [img][D], compact (slot w - 1 of the record)
    const Relax *tab;
    long tab_ld;
    float *gout;           // G_bar_{m+1} (nullable at the last layer)
    float *gc;             // [img][D] compact: alpha-gradient contributions (k_alpha_grad)
    float *gbeta;          // [nnz][rpi] beta-gradient of first split entries (nullable)
    int hw;                // H*W of layer m (C-major index)
    int rpi;
    float rrpi;
};

struct FwdParams {         // z_m = W_m h_{m-1} + b_m for sample rows
    float *out;            // z_m [img][D]
    const float *bias;     // b_m per channel
    long D;
};

// ----- product launchers ---------------------------------------------------------
// A plan picks the kernel of one product: path 0 = automatic (direct convolution when
// the geometry fits, else the implicit GEMM with the default tile), 1 = direct
// convolution with channel chunk cc (0 = largest that fits), 2 = implicit GEMM with tile
// configuration cfg (see gemm_candidates).
struct Plan {
    int path = 0;
    int cfg = -1;
    int cc = 0;
};
constexpr int kMaxCandidates = 32;

hipError_t gemm_relax(const GeomSet &gs, const float *A, long n_img, const RelaxParams &p,
                      hipStream_t st, const Plan &plan);
hipError_t gemm_conc(const GeomSet &gs, const float *A, long n_img, const ConcParams &p,
                     hipStream_t st, const Plan &plan);
hipError_t gemm_adj(const GeomSet &gs, const float *A, long n_img, const AdjParams &p,
                    hipStream_t st, const Plan &plan);
hipError_t gemm_fwd(const GeomSet &gs, const float *A, long n_img, const FwdParams &p,
                    hipStream_t st, const Plan &plan);
// Valid plans for a product (direct variants first, then GEMM tiles); returns the count.
int plan_candidates(const GeomSet &gs, Plan *out, int cap);
// gemm.hip: implicit GEMM with an explicit tile configuration (cfg < 0: default)
hipError_t gemm_relax_cfg(const GeomSet &gs, const float *A, long n_img, const RelaxParams &p,
                          hipStream_t st, int cfg);
hipError_t gemm_conc_cfg(const GeomSet &gs, const float *A, long n_img, const ConcParams &p,
                         hipStream_t st, int cfg);
hipError_t gemm_adj_cfg(const GeomSet &gs, const float *A, long n_img, const AdjParams &p,
                        hipStream_t st, int cfg);
hipError_t gemm_fwd_cfg(const GeomSet &gs, const float *A, long n_img, const FwdParams &p,
                        hipStream_t st, int cfg);
int gemm_candidates(const GeomSet &gs, int *cfgs, int cap);
// conv.hip: direct convolution (cc = 0: largest chunk that fits; mode 1 or 3: tiles staged
// by LDS DMA, else through registers; mode 2 or 3: 16x16 MFMA tiles for 32 output
// channels); *used = false when the geometry does not fit
hipError_t direct_relax(const GeomSet &gs, const float *A, long n_img, const RelaxParams &p,
                        hipStream_t st, int cc, int mode, bool *used);
hipError_t direct_conc(const GeomSet &gs, const float *A, long n_img, const ConcParams &p,
                       hipStream_t st, int cc, int mode, bool *used);
hipError_t direct_adj(const GeomSet &gs, const float *A, long n_img, const AdjParams &p,
                      hipStream_t st, int cc, int mode, bool *used);
hipError_t direct_fwd(const GeomSet &gs, const float *A, long n_img, const FwdParams &p,
                      hipStream_t st, int cc, int mode, bool *used);
int direct_candidates(const GeomSet &gs, int *cc, int *mode, int cap);

// ----- auxiliary kernels (aux.hip) ---------------------------------------------------
struct LayerShape {        // output shape of a ReLU layer (for index maps)
    int C, HW;             // channels, pixels
    long off;              // offset in the flat ReLU index
    long d;
};

constexpr int MAX_RELU_LAYERS = 128;

// The ReLU layers' shapes on the host (l) and in device memory (dev), with the device
// prefix sums of the relaxation-table tiles per layer (tile0[m] = tiles of layers < m).
struct NetShapes {
    int n;                 // number of ReLU layers described
    LayerShape l[MAX_RELU_LAYERS];
    const LayerShape *dev;
    const int32_t *tile0;
};
// Tiles of the relaxation-table kernel for one ReLU layer (host and device).
constexpr int PREP_TILE = 1024;
__host__ __device__ inline int prep_tiles(const LayerShape &L) {
    if (L.HW == 1) return (int)((L.d + PREP_TILE - 1) / PREP_TILE);
    if (L.C > PREP_TILE) return L.HW * ((L.C + PREP_TILE - 1) / PREP_TILE);
    const int P = PREP_TILE / L.C;
    return (L.HW + P - 1) / P;
}

hipError_t launch_fill(float *p, long n, float v, hipStream_t st);
// deterministic row sums: s[img] += the slots' first values, mag[img] += their second
// values, each summed in slot order (one wave per img, a fixed shuffle tree)
hipError_t launch_det_reduce(long n_img, long nslot, const float *part, float *s, float *mag,
                             hipStream_t st);
// cnt[0] += NaN count, cnt[1] += Inf count of p[0 .. n) (debug checks)
hipError_t launch_count_nonfinite(const float *p, long n, int32_t *cnt, hipStream_t st);
hipError_t launch_prep_tables(const NetShapes &ns, int n_layers_used, int n_inst,
                              long n_relu, const float *lo, const float *hi,
                              const int32_t *bound_of, const float *alpha, Relax *tab,
                              int32_t *infeas, int n_bounds, int32_t *slot, int32_t *slot_inv,
                              int32_t *slot_count, int32_t *srow, int max_rows, hipStream_t st);
// alpha-gradient of one layer from the compact per-row contributions gc (sum over an
// instance's rows per slot, written C-major), then 0 at the layer's split neurons
hipError_t launch_alpha_grad(int n_inst, int rows, long D, const LayerShape &L, int layer,
                             long n_relu, const int32_t *srow, const int32_t *slot_count,
                             const int32_t *slot_inv, const float *gc, float *galpha, long ga_ld,
                             long ga_off, int nnz, const int32_t *sp_inst, const int32_t *sp_layer,
                             const int32_t *sp_j, hipStream_t st);
hipError_t launch_prep_splits(const NetShapes &ns, int n_layers_used, int n_inst, long n_relu,
                              const float *lo, const float *hi, const int32_t *bound_of,
                              const int32_t *off, const int32_t *idx, const int8_t *sign,
                              Relax *tab, int32_t *infeas, int32_t *sp_inst,
                              int32_t *sp_layer, int32_t *sp_j, int32_t *sp_dup, int n_bounds,
                              int stop_m, int stop_relu, float *stop_cen, float *stop_rad,
                              hipStream_t st);
hipError_t launch_prep_stop_box(int n_inst, const LayerShape &L, long n_relu, const float *lo,
                                const float *hi, const int32_t *bound_of, int n_bounds, bool relu,
                                float *cen, float *rad, hipStream_t st);
hipError_t launch_box_conc(long img0, long n_img, int rpi, long D, const float *lam, const float *cen,
                           const float *rad, float *low, float *mag, float *save, hipStream_t st);
hipError_t launch_adj_stop_linear(long n_img, int rows, long D, const float *lam, const float *g,
                                  const float *cen, const float *rad, const float *gl,
                                  const int32_t *infeas, float *sbar, const Relax *tab, long tab_ld,
                                  float *gout, float *gc, int C, int HW, hipStream_t st);
hipError_t launch_beta_grad_stop(int nnz, int rows, int layer, long D, const int32_t *sp_inst,
                                 const int32_t *sp_layer, const int32_t *sp_j, const int8_t *sign,
                                 const float *lam, const float *cen, const float *rad,
                                 const float *sbar, float *gbeta, hipStream_t st);
hipError_t launch_prep_box(int n_inst, int C0, int HW0, const float *x_lo, const float *x_hi,
                           float *cen, float *rad, hipStream_t st);
hipError_t launch_init_spec(long img0, long n_img, int rows, int rpi, const float *spec,
                            long dk, int Ck, int HWk, const float *bias_k, float *lam,
                            float *s, float *mag, float *low, hipStream_t st);

struct IdentityParams {
    // target layer k
    int kind;                  // 0 linear, 1 conv
    const float *W;            // user weight of layer k (C-major)
    const float *bias_k;
    int ci, hi_, wi;           // input shape of layer k
    int co, ho, wo;            // output shape of layer k
    int kh, kw, stride, pad;
    long dk, din;              // widths of z_k and of the layer's input
    int rpi;                   // 2*dk (both sides) or dk
    long img0;
    // relax mode (k > 1): table and bias of layer k-1
    const Relax *tab;
    long tab_ld;
    const float *bias_m;
    int chan_m;
    float *out;                // Lambda_{k-1} [img][din]
    const float *bsum;         // split-multiplier terms (see RelaxParams), nullable
    // concretise mode (k == 1)
    const float *cen, *rad;
    float *emit;
    // accumulators
    float *s, *mag, *low;
};
hipError_t launch_init_identity(const IdentityParams &p, long n_img, bool conc, hipStream_t st);

// Per first split entry q and row r: sum over the instance's entries on the same neuron
// of sign * beta (the term the relaxation epilogue subtracts at the split neuron).
hipError_t launch_beta_sum(int nnz, int rows, const int32_t *off, const int32_t *idx,
                           const int8_t *sign, const int32_t *sp_inst, const int32_t *sp_layer,
                           const int32_t *sp_dup, const float *beta, float *bsum, hipStream_t st);
hipError_t launch_finalize(long img0, long n_img, int rows, int rpi, const float *s,
                           const float *low, const float *mag, const int32_t *infeas,
                           bool slack, float *lower, float *upper, long ld, float *offset,
                           float *offset_mag, float *best, float *best_upper, hipStream_t st);
hipError_t launch_adj_init(long n_img, int rows, long d0, const float *gl, const float *g1,
                           const float *cen, const float *rad, const int32_t *infeas,
                           float *gbar, float *sbar, hipStream_t st);

struct BetaGradLayer {         // layer m, for the split-multiplier gradient
    int kind;
    const float *W;            // user weight (C-major)
    const float *bias;
    int ci, hi_, wi, co, ho, wo, kh, kw, stride, pad;
    long din, dout;
};
hipError_t launch_beta_grad(int nnz, int rows, int layer, const BetaGradLayer &L,
                            const int32_t *sp_inst, const int32_t *sp_layer,
                            const int32_t *sp_j, const int32_t *sp_dup, const int8_t *sign,
                            const float *gbar_m, const float *gl, const int32_t *infeas,
                            float *gbeta, hipStream_t st);
hipError_t launch_to_internal(long n_img, int C, int HW, const float *x, float *y, hipStream_t st);
hipError_t launch_sample_minmax(long n_sub, int per_sub, long D, int C, int HW, float *z,
                                float *lo, float *hi, long ld, bool relu, float *out, bool merge,
                                hipStream_t st);
hipError_t launch_adam(long n, float *p, const float *g, float *m, float *v, int step,
                       float lr, float b1, float b2, float eps, float gs, float lo, float hi,
                       hipStream_t st);
// Adam constants of one step (bias corrections folded in on the host)
struct AdamArgs {
    float b1, b2, bc1, bc2s, lr, eps, gs, lo, hi;
};
AdamArgs adam_args(int step, float lr, float b1, float b2, float eps, float gs, float lo, float hi);
// alpha-gradient of one ReLU layer fused with the Adam step on alpha (moments in slot
// order); clears split neurons' slots of gc first
hipError_t launch_alpha_adam(int n_inst, int rows, long D, const LayerShape &L, int layer,
                             long n_relu, const int32_t *srow, const int32_t *slot_count,
                             const int32_t *slot_inv, const int32_t *slot, float *gc, float *alpha,
                             float *m, float *v, long ld, long aoff, int nnz,
                             const int32_t *sp_inst, const int32_t *sp_layer, const int32_t *sp_j,
                             const AdamArgs &a, hipStream_t st);
hipError_t launch_concretize(int n_inst, int rows, long d0, const float *coeff,
                             const float *offset, const float *offset_mag, const float *x_lo,
                             const float *x_hi, bool slack, float *lower, hipStream_t st);

// Packing helpers (aux.hip)
hipError_t launch_pack_T(const float *W, int kind, int ci, int hi_, int wi, int co, int ho,
                         int wo, int kh, int kw, int stride, int pad, int py, int px, int ky0,
                         int kx0, int Ty, int Tx, int N, int K, int Kp, int Np, float *Bt,
                         hipStream_t st);
hipError_t launch_pack_F(const float *W, int kind, int ci, int hi_, int wi, int co, int kh,
                         int kw, int N, int K, int Kp, int Np, float *Bt, hipStream_t st);

constexpr float KAPPA_U = 64.0f / 16777216.0f;   // slack factor: 64 * 2^-24

}  // namespace bp
