// Host side of the C ABI declared in include/bound.h: layer validation, weight packing,
// workspace management, the layer-by-layer schedule of a backward bound pass (Theorem 1
// with Lemma 1 and Theorem 2 of the paper's Appendix B), its adjoint, and Adam.
#include "../../include/bound.h"
#include "bound_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

using namespace bp;

namespace {

thread_local std::string g_err;

bound_status fail(bound_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail(BOUND_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));      \
    } while (0)

inline long roundup(long x, long m) { return (x + m - 1) / m * m; }

struct LayerInfo {
    bound_layer L;
    long din, dout;
    GeomSet gT;  // backward product Lambda W (transposed convolution for Conv2d)
    GeomSet gF;  // forward product (adjoint pass)
};

}  // namespace

struct bound_net {
    int n_layers = 0;
    std::vector<LayerInfo> layers;   // index 0 = layer 1
    std::vector<long> d;             // d_0 .. d_L
    long n_relu = 0;
    NetShapes ns{};                  // ReLU layers z_1 .. z_{L-1}
    int C0 = 0, HW0 = 0;             // input shape
    int max_inst = 0;
    long max_rows = 0, max_save_rows = 0, max_d = 0;
    std::vector<void *> allocs;
    float *buf[2] = {nullptr, nullptr};
    float *acc_s = nullptr, *acc_mag = nullptr, *acc_low = nullptr;
    Relax *tab = nullptr;
    int32_t *slot = nullptr;         // compact save slots of the unstable neurons per bound row
    int32_t *slot_inv = nullptr;     // slot -> internal neuron index, per bound row
    int32_t *slot_count = nullptr;   // unstable neurons per (bound row, ReLU layer)
    int32_t *srow = nullptr;         // bound row of each instance
    float *gcbuf = nullptr;          // per-img alpha-gradient contributions of one layer
    int32_t *infeas = nullptr;
    float *cen = nullptr, *rad = nullptr;
    float *save = nullptr;
    float *sbar = nullptr;
    float *stop_cen = nullptr, *stop_rad = nullptr;  // early-stop node box [max_inst][max relu width]
    float *zeros = nullptr;                         // [max channels]: "no bias" at a linear stop
    long max_relu_d = 0, max_chan = 0;
    int32_t *sp = nullptr;           // 4 x sp_cap: instance, layer, internal index, repeated entry
    int8_t *sp_sign = nullptr;
    long sp_cap = 0;
    float *bsum = nullptr;           // [nnz][rows]: split-multiplier term per first entry
    long bsum_cap = 0;
    int32_t *dbg = nullptr;          // [2] NaN / Inf counts of the debug checks
    float *det_part = nullptr;       // deterministic row-sum slots (BOUND_OPT_DETERMINISTIC)
    long det_cap = 0;                // slots per img it holds
    int options = 0;
    // kernel plan per product (key: 'R'/'C'/'A' * 256 + layer), chosen by bound_autotune
    std::map<int, Plan> plans;
    bool tuning = false;
    std::string tune_report;
    // per-launch timing
    bool prof = false;
    struct ProfRec { std::string label; hipEvent_t a, b; };
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    // state of the last SAVE_FOR_GRAD pass
    bool saved = false;
    int64_t pass_seq = 0;            // id of the last SAVE_FOR_GRAD pass (1, 2, ...)
    int s_target = 0, s_rows = 0, s_n_inst = 0, s_nnz = 0, s_nnz_arg = 0, s_stop = 0, s_mode = 0;
    std::vector<long> s_off;         // offset of saved G_m (m = 1..k) in the save buffer
    long s_lam_off = 0;              // saved Lambda at a linear early stop
    // checkpointed mode: Lambda_t kept at checkpoint products t (offsets), every c-th
    // product from the top; the adjoint recomputes a segment's G from its checkpoint
    // into the segment area (c layers, each total x max_relu_d)
    bool s_recompute = false, s_inject = false;
    int s_c = 1;
    std::vector<long> s_ck;          // offset of Lambda_t, or -1 if t is not a checkpoint
    long s_seg_off = 0;
    float *rbuf = nullptr;           // ping-pong scratch of the recomputation
    long rbuf_cap = 0;

    ~bound_net() {
        for (auto &r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
        for (hipEvent_t e : pool) hipEventDestroy(e);
        for (void *p : allocs) hipFree(p);
    }
    hipEvent_t event() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        hipEventCreate(&e);
        return e;
    }
    template <class T> bool alloc(T **p, long n) {
        void *q = nullptr;
        if (n <= 0) n = 1;
        if (hipMalloc(&q, sizeof(T) * (size_t)n) != hipSuccess) return false;
        allocs.push_back(q);
        *p = (T *)q;
        return true;
    }
    const float *bias(int m) const { return layers[m - 1].L.bias; }        // b_m
    int chan(int m) const { return layers[m - 1].L.out_c; }                // channels of z_m
    long relu_off(int m) const { return ns.l[m - 1].off; }                 // offset of z_m
};

namespace {

// Brackets the launches issued in its scope with events on the launch stream when the
// handle's profiler is on and the stream is not being captured.
struct ProfScope {
    bound_net *net;
    hipStream_t st;
    hipEvent_t a = nullptr;
    std::string label;
    ProfScope(bound_net *n, hipStream_t s, std::string l) : net(n), st(s), label(std::move(l)) {
        if (!net->prof) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        a = net->event();
        if (a && hipEventRecord(a, st) != hipSuccess) { net->pool.push_back(a); a = nullptr; }
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = net->event();
        if (b && hipEventRecord(b, st) == hipSuccess) net->recs.push_back({label, a, b});
        else { net->pool.push_back(a); if (b) net->pool.push_back(b); }
    }
};

// Run one product with its plan.  In tuning mode, time every valid candidate on the
// live inputs (3 launches each after one warm-up; the product is re-run, so the pass's
// accumulators are scratch until the normal pass that follows tuning) and keep the
// fastest.
template <class F>
bound_status run_product(bound_net *net, hipStream_t st, int key, const GeomSet &gs, F launch) {
    if (!net->tuning) {
        Plan p;
        if (net->options & BOUND_OPT_GEMM_ONLY) {
            p.path = 2;
        } else {
            auto it = net->plans.find(key);
            if (it != net->plans.end())
                p = it->second;
            else if (net->options & BOUND_OPT_DIRECT_DMA)
                p.cfg = 1;
        }
        HIPCHK(launch(p));
        return BOUND_OK;
    }
    Plan cand[kMaxCandidates];
    const int nc = plan_candidates(gs, cand, kMaxCandidates);
    hipEvent_t a = net->event(), b = net->event();
    float best = INFINITY;
    Plan bestp;
    char line[160];
    for (int c = 0; c < nc; ++c) {
        HIPCHK(launch(cand[c]));
        HIPCHK(hipEventRecord(a, st));
        for (int r = 0; r < 3; ++r) HIPCHK(launch(cand[c]));
        HIPCHK(hipEventRecord(b, st));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        ms /= 3.f;
        std::snprintf(line, sizeof line, "%c%d %s cfg=%d cc=%d %.4f ms\n", (char)(key >> 8), key & 255,
                      cand[c].path == 1 ? "direct" : "gemm", cand[c].cfg, cand[c].cc, ms);
        net->tune_report += line;
        if (ms < best) {
            best = ms;
            bestp = cand[c];
        }
    }
    net->pool.push_back(a);
    net->pool.push_back(b);
    if (nc > 0) net->plans[key] = bestp;
    HIPCHK(launch(bestp));
    return BOUND_OK;
}

inline int pkey(char c, int m) { return ((int)c << 8) | m; }

// Row-sum slots per img of the relaxation / concretisation product of layer m: its
// output pixels (width / N) times ceil(N / 16) column groups, N the product's columns.
long det_slots(const bound_net *net, int m) {
    const int N = net->layers[m - 1].gT.g[0].N;
    const long D = net->d[m - 1];
    return N > 0 ? (D / N) * ((N + 15) / 16) : 1;
}

// With BOUND_OPT_DETERMINISTIC: the zeroed slots of the product of layer m for n_img imgs
// (det.part stays null otherwise: float atomics).
bound_status det_begin(bound_net *net, hipStream_t st, int m, long n_img, DetSums &det) {
    det = DetSums{};
    if (!(net->options & BOUND_OPT_DETERMINISTIC)) return BOUND_OK;
    det.nslot = det_slots(net, m);
    const int N = net->layers[m - 1].gT.g[0].N;
    det.ncu = (N + 15) / 16;
    if (!net->det_part || det.nslot > net->det_cap)
        return fail(BOUND_E_STATE, "deterministic row sums: slots not allocated");
    det.part = net->det_part;
    HIPCHK(launch_fill(det.part, n_img * det.nslot * 2, 0.f, st));
    return BOUND_OK;
}

// BOUND_OPT_CHECK: count the NaN / Inf values of n floats at p (a product's output) and
// fail with BOUND_E_NUMERIC naming `what` if there are any.  Synchronises the stream;
// skipped while the stream is being captured.
bound_status debug_check(bound_net *net, hipStream_t st, const float *p, long n, const std::string &what) {
    if (!(net->options & BOUND_OPT_CHECK) || !p || n <= 0) return BOUND_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return BOUND_OK;
    int32_t h[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(net->dbg, h, sizeof h, hipMemcpyHostToDevice, st));
    HIPCHK(launch_count_nonfinite(p, n, net->dbg, st));
    HIPCHK(hipMemcpyAsync(h, net->dbg, sizeof h, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h[0] || h[1])
        return fail(BOUND_E_NUMERIC, what + ": " + std::to_string(h[0]) + " NaN and " +
                                         std::to_string(h[1]) + " Inf values");
    return BOUND_OK;
}

std::string lbl(const char *f, int m) {
    char buf[48];
    std::snprintf(buf, sizeof buf, f, m);
    return buf;
}

bound_status build_geoms(bound_net *net, hipStream_t st) {
    for (int i = 0; i < net->n_layers; ++i) {
        LayerInfo &li = net->layers[i];
        const bound_layer &L = li.L;
        if (L.kind == BOUND_LINEAR) {
            Geom t{};
            t.H = t.W = 1; t.C = (int)li.dout; t.OH = t.OW = 1; t.kh = t.kw = 1; t.stride = 1;
            t.K = (int)li.dout; t.N = (int)li.din; t.Kp = (int)roundup(li.dout, 16);
            t.DH = t.DW = 1; t.ostr = 1;
            const long NpT = roundup(li.din, 128);
            float *bt;
            if (!net->alloc(&bt, NpT * t.Kp)) return fail(BOUND_E_NOMEM, "weight packing");
            HIPCHK(launch_pack_T(L.weight, 0, L.in_c, L.in_h, L.in_w, L.out_c, 1, 1, 1, 1, 1, 0, 0, 0,
                                 0, 0, 1, 1, t.N, t.K, t.Kp, (int)NpT, bt, st));
            t.Bt = bt;
            set_recips(t);
            li.gT.g[0] = t; li.gT.n = 1;

            Geom f{};
            f.H = f.W = 1; f.C = (int)li.din; f.OH = f.OW = 1; f.kh = f.kw = 1; f.stride = 1;
            f.K = (int)li.din; f.N = (int)li.dout; f.Kp = (int)roundup(li.din, 16);
            f.DH = f.DW = 1; f.ostr = 1;
            const long NpF = roundup(li.dout, 128);
            float *bf;
            if (!net->alloc(&bf, NpF * f.Kp)) return fail(BOUND_E_NOMEM, "weight packing");
            HIPCHK(launch_pack_F(L.weight, 0, L.in_c, L.in_h, L.in_w, L.out_c, 1, 1, f.N, f.K, f.Kp,
                                 (int)NpF, bf, st));
            f.Bt = bf;
            set_recips(f);
            li.gF.g[0] = f; li.gF.n = 1;
        } else {
            // forward convolution (adjoint)
            Geom f{};
            f.H = L.in_h; f.W = L.in_w; f.C = L.in_c; f.OH = L.out_h; f.OW = L.out_w;
            f.kh = L.kh; f.kw = L.kw; f.stride = L.stride; f.pad_y = f.pad_x = L.pad;
            f.K = L.kh * L.kw * L.in_c; f.N = L.out_c; f.Kp = (int)roundup(f.K, 16);
            f.DH = L.out_h; f.DW = L.out_w; f.ostr = 1;
            const long NpF = roundup(f.N, 128);
            float *bf;
            if (!net->alloc(&bf, NpF * f.Kp)) return fail(BOUND_E_NOMEM, "weight packing");
            HIPCHK(launch_pack_F(L.weight, 1, L.in_c, L.in_h, L.in_w, L.out_c, L.kh, L.kw, f.N, f.K,
                                 f.Kp, (int)NpF, bf, st));
            f.Bt = bf;
            set_recips(f);
            li.gF.g[0] = f; li.gF.n = 1;
            // transposed convolution, one stride-1 implicit GEMM per output phase
            const int s = L.stride;
            int np = 0;
            for (int py = 0; py < s; ++py) {
                for (int px = 0; px < s; ++px) {
                    const int ky0 = (py + L.pad) % s, kx0 = (px + L.pad) % s;
                    const int Ty = ky0 < L.kh ? (L.kh - ky0 + s - 1) / s : 0;
                    const int Tx = kx0 < L.kw ? (L.kw - kx0 + s - 1) / s : 0;
                    const int Ay = (L.in_h - py + s - 1) / s, Ax = (L.in_w - px + s - 1) / s;
                    if (Ay <= 0 || Ax <= 0) continue;
                    const int dy = (py + L.pad - ky0) / s, dx = (px + L.pad - kx0) / s;
                    Geom t{};
                    t.H = L.out_h; t.W = L.out_w; t.C = L.out_c;
                    t.OH = Ay; t.OW = Ax;
                    t.kh = Ty; t.kw = Tx; t.stride = 1;
                    t.pad_y = Ty - 1 - dy; t.pad_x = Tx - 1 - dx;
                    t.K = Ty * Tx * L.out_c; t.N = L.in_c; t.Kp = (int)roundup(t.K > 0 ? t.K : 1, 16);
                    t.DH = L.in_h; t.DW = L.in_w; t.ostr = s; t.oy0 = py; t.ox0 = px;
                    const long NpT = roundup(t.N, 128);
                    float *bt;
                    if (!net->alloc(&bt, NpT * t.Kp)) return fail(BOUND_E_NOMEM, "weight packing");
                    HIPCHK(launch_pack_T(L.weight, 1, L.in_c, L.in_h, L.in_w, L.out_c, L.out_h,
                                         L.out_w, L.kh, L.kw, s, L.pad, py, px, ky0, kx0, Ty, Tx,
                                         t.N, t.K, t.Kp, (int)NpT, bt, st));
                    t.Bt = bt;
                    set_recips(t);
                    li.gT.g[np++] = t;
                }
            }
            li.gT.n = np;
        }
    }
    return BOUND_OK;
}

// Scratch for the split list (nnz entries) and, with beta, its per-row multiplier terms
// (nnz x rows).  Grows only outside stream capture; old buffers stay until bound_destroy.
bound_status ensure_split_cap(bound_net *net, long nnz, long rows, hipStream_t st) {
    const bool grow_sp = nnz > net->sp_cap, grow_b = nnz * rows > net->bsum_cap;
    if (!grow_sp && !grow_b) return BOUND_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(BOUND_E_NOMEM, "split list larger than any earlier pass while the stream is "
                                   "being captured; run one pass of this size before capturing");
    if (grow_sp) {
        const long cap = roundup(nnz, 4096);
        int32_t *sp;
        int8_t *sg;
        if (!net->alloc(&sp, 4 * cap) || !net->alloc(&sg, cap))
            return fail(BOUND_E_NOMEM, "split scratch");
        net->sp = sp;
        net->sp_sign = sg;
        net->sp_cap = cap;
    }
    if (grow_b) {
        const long cap = roundup(nnz * rows, 4096);
        float *b;
        if (!net->alloc(&b, cap)) return fail(BOUND_E_NOMEM, "split multiplier scratch");
        net->bsum = b;
        net->bsum_cap = cap;
    }
    return BOUND_OK;
}

}  // namespace

extern "C" {

const char *bound_last_error(void) { return g_err.c_str(); }

bound_status bound_init(const bound_layer *layers, int32_t n_layers, int32_t max_inst,
                        int64_t max_rows, int64_t max_save_rows, void *stream, bound_net **out) {
    if (!layers || !out || n_layers < 1 || n_layers > MAX_RELU_LAYERS + 1 || max_inst < 1 ||
        max_rows < 1 || max_save_rows < 0 || max_save_rows > max_rows)
        return fail(BOUND_E_ARG, "bound_init: bad arguments (need 1 <= n_layers <= " +
                                     std::to_string(MAX_RELU_LAYERS + 1) +
                                     ", max_inst >= 1, 0 <= max_save_rows <= max_rows)");
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    auto *net = new bound_net();
    net->n_layers = n_layers;
    net->max_inst = max_inst;
    net->max_rows = max_rows;
    net->max_save_rows = max_save_rows;
    net->layers.resize(n_layers);
    for (int i = 0; i < n_layers; ++i) {
        const bound_layer &L = layers[i];
        LayerInfo &li = net->layers[i];
        li.L = L;
        if (!L.weight || !L.bias) {
            delete net;
            return fail(BOUND_E_ARG, "layer " + std::to_string(i + 1) + ": null weight or bias");
        }
        if (L.kind == BOUND_LINEAR) {
            if (L.in_c < 1 || L.in_h < 1 || L.in_w < 1 || L.out_c < 1 || L.out_h != 1 || L.out_w != 1) {
                delete net;
                return fail(BOUND_E_SHAPE, "linear layer " + std::to_string(i + 1) + ": bad shape");
            }
        } else if (L.kind == BOUND_CONV2D) {
            const bool ok = L.in_c >= 1 && L.in_h >= 1 && L.in_w >= 1 && L.out_c >= 1 &&
                            L.kh >= 1 && L.kh == L.kw && L.stride >= 1 && L.stride <= 2 &&
                            L.pad >= 0 && L.out_h == (L.in_h + 2 * L.pad - L.kh) / L.stride + 1 &&
                            L.out_w == (L.in_w + 2 * L.pad - L.kw) / L.stride + 1 && L.out_h >= 1 &&
                            L.out_w >= 1;
            if (!ok) {
                delete net;
                return fail(BOUND_E_SHAPE, "conv layer " + std::to_string(i + 1) +
                                               ": bad shape (square kernel, stride 1 or 2, "
                                               "out = (in + 2 pad - k) / stride + 1)");
            }
            if (L.kh * L.kw * L.in_c > 1024 || L.kh * L.kw * L.out_c > 1024) {
                delete net;
                return fail(BOUND_E_SHAPE, "conv layer " + std::to_string(i + 1) +
                                               ": kh*kw*channels must not exceed 1024");
            }
        } else {
            delete net;
            return fail(BOUND_E_ARG, "layer " + std::to_string(i + 1) + ": unknown kind");
        }
        li.din = (long)L.in_c * L.in_h * L.in_w;
        li.dout = (long)L.out_c * L.out_h * L.out_w;
        if (i > 0) {
            const bound_layer &P = layers[i - 1];
            if (P.out_c != L.in_c || P.out_h != L.in_h || P.out_w != L.in_w) {
                delete net;
                return fail(BOUND_E_SHAPE, "layer " + std::to_string(i + 1) +
                                               ": input shape differs from the output of layer " +
                                               std::to_string(i));
            }
        }
    }
    net->d.push_back(net->layers[0].din);
    for (auto &li : net->layers) net->d.push_back(li.dout);
    net->C0 = layers[0].in_c;
    net->HW0 = layers[0].in_h * layers[0].in_w;
    net->ns.n = n_layers - 1;
    long off = 0;
    for (int t = 0; t < n_layers - 1; ++t) {
        const bound_layer &L = layers[t];
        net->ns.l[t].C = L.out_c;
        net->ns.l[t].HW = L.out_h * L.out_w;
        net->ns.l[t].off = off;
        net->ns.l[t].d = net->d[t + 1];
        off += net->d[t + 1];
    }
    net->n_relu = off;
    net->max_d = 0;
    for (long x : net->d) net->max_d = x > net->max_d ? x : net->max_d;
    net->max_relu_d = 1;
    net->max_chan = 1;
    for (int t = 0; t < n_layers - 1; ++t)
        net->max_relu_d = net->d[t + 1] > net->max_relu_d ? net->d[t + 1] : net->max_relu_d;
    for (int i = 0; i < n_layers; ++i)
        net->max_chan = layers[i].out_c > net->max_chan ? layers[i].out_c : net->max_chan;

    bool ok = net->alloc(&net->buf[0], max_rows * net->max_d) &&
              net->alloc(&net->buf[1], max_rows * net->max_d) &&
              net->alloc(&net->acc_s, max_rows) && net->alloc(&net->acc_mag, max_rows) &&
              net->alloc(&net->acc_low, max_rows) &&
              net->alloc(&net->tab, (long)max_inst * (net->n_relu > 0 ? net->n_relu : 1)) &&
              net->alloc(&net->slot, (long)max_inst * (net->n_relu > 0 ? net->n_relu : 1)) &&
              net->alloc(&net->slot_inv, (long)max_inst * (net->n_relu > 0 ? net->n_relu : 1)) &&
              net->alloc(&net->slot_count, (long)max_inst * MAX_RELU_LAYERS) &&
              net->alloc(&net->srow, (long)max_inst) &&
              net->alloc(&net->gcbuf, max_save_rows * (net->max_relu_d > 0 ? net->max_relu_d : 1)) &&
              net->alloc(&net->infeas, max_inst) && net->alloc(&net->cen, (long)max_inst * net->d[0]) &&
              net->alloc(&net->rad, (long)max_inst * net->d[0]) &&
              net->alloc(&net->sbar, max_save_rows > 0 ? max_save_rows : 1) &&
              net->alloc(&net->save, max_save_rows * (net->d[0] + net->n_relu + net->max_relu_d)) &&
              net->alloc(&net->stop_cen, (long)max_inst * net->max_relu_d) &&
              net->alloc(&net->stop_rad, (long)max_inst * net->max_relu_d) &&
              net->alloc(&net->zeros, net->max_chan);
    LayerShape *dls = nullptr;
    int32_t *dt0 = nullptr;
    ok = ok && net->alloc(&dls, n_layers) && net->alloc(&dt0, n_layers + 1) &&
         net->alloc(&net->dbg, 2);
    {
        const char *e = std::getenv("BOUND_DEBUG");
        if (e && e[0] && e[0] != '0') net->options |= BOUND_OPT_CHECK;
    }
    if (!ok) {
        delete net;
        return fail(BOUND_E_NOMEM, "bound_init: workspace allocation failed");
    }
    // the layer shapes and the relaxation-table tile prefix in device memory
    {
        std::vector<int32_t> t0(n_layers + 1, 0);
        for (int t = 0; t < net->ns.n; ++t) t0[t + 1] = t0[t] + prep_tiles(net->ns.l[t]);
        if (hipMemcpyAsync(dls, net->ns.l, sizeof(LayerShape) * (size_t)(net->ns.n > 0 ? net->ns.n : 1),
                           hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(dt0, t0.data(), sizeof(int32_t) * t0.size(), hipMemcpyHostToDevice, st) !=
                hipSuccess) {
            delete net;
            return fail(BOUND_E_HIP, "bound_init: layer table upload");
        }
        net->ns.dev = dls;
        net->ns.tile0 = dt0;
        // the host vector must outlive the asynchronous copy
        if (hipStreamSynchronize(st) != hipSuccess) {
            delete net;
            return fail(BOUND_E_HIP, "bound_init: layer table upload");
        }
    }
    bound_status s = ensure_split_cap(net, (long)max_inst * 16, 0, st);
    if (s != BOUND_OK) { delete net; return s; }
    s = build_geoms(net, st);
    if (s != BOUND_OK) { delete net; return s; }
    if (launch_fill(net->zeros, net->max_chan, 0.f, st) != hipSuccess) {
        delete net;
        return fail(BOUND_E_HIP, "bound_init: fill");
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete net;
        return fail(BOUND_E_HIP, std::string("bound_init: ") + hipGetErrorString(e));
    }
    *out = net;
    return BOUND_OK;
}

bound_status bound_dims(const bound_net *net, int32_t *n_layers, int32_t *d, int32_t *n_relu) {
    if (!net) return fail(BOUND_E_ARG, "bound_dims: null net");
    if (n_layers) *n_layers = net->n_layers;
    if (d)
        for (size_t i = 0; i < net->d.size(); ++i) d[i] = (int32_t)net->d[i];
    if (n_relu) *n_relu = (int32_t)net->n_relu;
    return BOUND_OK;
}

bound_status bound_backward(bound_net *net, const bound_pass *P, const bound_out *out, void *stream) {
    if (!net || !P || !out) return fail(BOUND_E_ARG, "bound_backward: null argument");
    hipStream_t st = (hipStream_t)stream;
    const int L = net->n_layers;
    const int k = P->target;
    if (k < 1 || k > L) return fail(BOUND_E_ARG, "target must be in 1..n_layers");
    if (P->n_inst < 1 || P->n_inst > net->max_inst)
        return fail(BOUND_E_NOMEM, "n_inst must be in 1..max_inst");
    if (P->rows < 1) return fail(BOUND_E_ARG, "rows must be >= 1");
    const bool ident = P->spec == nullptr;
    const long dk = net->d[k];
    if (ident && P->rows != dk) return fail(BOUND_E_SHAPE, "identity spec needs rows == d_target");
    if (k > 1 && (!P->lo || !P->hi)) return fail(BOUND_E_ARG, "lo/hi required when target > 1");
    if (k > 1 && P->n_bounds < (P->bound_of ? 1 : P->n_inst))
        return fail(BOUND_E_ARG, "n_bounds too small");
    const bool both = (P->flags & BOUND_BOTH_SIDES) != 0;
    const bool save = (P->flags & BOUND_SAVE_FOR_GRAD) != 0;
    const bool slack = (P->flags & BOUND_NO_SLACK) == 0;
    const int nnz = P->nnz;
    if (nnz < 0 || nnz >= (1 << 24))    // split entries are numbered exactly in FP32
        return fail(BOUND_E_ARG, "nnz must be in [0, 2^24)");
    if (nnz > 0 && (!P->split_off || !P->split_idx || !P->split_sign))
        return fail(BOUND_E_ARG, "split arrays required when nnz > 0");
    if (P->beta && nnz == 0) return fail(BOUND_E_ARG, "beta given without splits");
    if (P->beta && both) return fail(BOUND_E_ARG, "beta cannot be combined with BOTH_SIDES");
    if ((P->x_lo == nullptr) != (P->x_hi == nullptr)) return fail(BOUND_E_ARG, "x_lo/x_hi: both or neither");
    const bool conc = P->x_lo != nullptr;
    if (conc && !out->lower) return fail(BOUND_E_ARG, "lower output required");
    if (conc && both && !out->upper) return fail(BOUND_E_ARG, "upper output required with BOTH_SIDES");
    if (!conc && (!out->coeff || !out->offset))
        return fail(BOUND_E_ARG, "coeff and offset outputs required without a box");
    const int rpi = P->rows * (both ? 2 : 1);
    const long total = (long)P->n_inst * rpi;
    if (save) {
        if (ident || !conc)
            return fail(BOUND_E_ARG, "SAVE_FOR_GRAD needs an explicit spec and a box");
        if (total > net->max_save_rows) return fail(BOUND_E_NOMEM, "n_inst*rows > max_save_rows");
    }
    const bool recompute = (P->flags & BOUND_RECOMPUTE) != 0;
    if (recompute && !save) return fail(BOUND_E_ARG, "BOUND_RECOMPUTE needs BOUND_SAVE_FOR_GRAD");
    if (recompute && P->stop_layer > 0)
        return fail(BOUND_E_ARG, "BOUND_RECOMPUTE is not combined with an early stop");
    const int sl = P->stop_layer, smode = sl > 0 ? P->stop_mode : 0;
    if (sl < 0 || (sl > 0 && (sl >= k || (smode != BOUND_STOP_RELU && smode != BOUND_STOP_LINEAR))))
        return fail(BOUND_E_ARG, "stop_layer must be 0 or in 1..target-1 with a stop_mode");
    if (sl > 0 && !conc) return fail(BOUND_E_ARG, "early stop needs x_lo/x_hi (coefficient output is on x)");
    const long ld = out->ld > 0 ? out->ld : P->rows;
    net->saved = false;
    // Bottom of the backward chain: the product of layer conc_m gets the concretising
    // epilogue (input box, or the ReLU-node box at a ReLU stop); relax_low is the lowest
    // product with the relaxation epilogue; at a linear stop the relaxed coefficients on
    // z_sl are concretised by a separate reduction.
    const int conc_m = smode == BOUND_STOP_LINEAR ? -1 : (smode == BOUND_STOP_RELU ? sl + 1 : 1);
    const int relax_low = smode == BOUND_STOP_LINEAR ? sl + 1 : (smode == BOUND_STOP_RELU ? sl + 2 : 2);
    const LayerShape *SL = sl > 0 ? &net->ns.l[sl - 1] : nullptr;

    // Relaxation tables (Lemma 1) for z_1 .. z_{k-1}, split clamping, box.
    const int used = k - 1;
    const bool inject = P->beta != nullptr && used > 0;
    if (nnz > 0) {
        bound_status s = ensure_split_cap(net, nnz, inject ? P->rows : 0, st);
        if (s != BOUND_OK) return s;
    }
    int32_t *sp_inst = net->sp, *sp_layer = net->sp + net->sp_cap, *sp_j = net->sp + 2 * net->sp_cap;
    int32_t *sp_dup = net->sp + 3 * net->sp_cap;
    const long d0 = net->d[0];
    {
    ProfScope prof_prep(net, st, "prep");
    if (used > 0) {
        HIPCHK(launch_prep_tables(net->ns, used, P->n_inst, net->n_relu, P->lo, P->hi, P->bound_of,
                                  P->alpha, net->tab, net->infeas, P->n_bounds, net->slot,
                                  net->slot_inv, net->slot_count, net->srow, net->max_inst, st));
    } else {
        HIPCHK(launch_fill((float *)net->infeas, P->n_inst, 0.f, st));
    }
    if (nnz > 0 && used > 0) {
        if (sl > 0)
            HIPCHK(launch_prep_stop_box(P->n_inst, *SL, net->n_relu, P->lo, P->hi, P->bound_of,
                                        P->n_bounds, smode == BOUND_STOP_RELU, net->stop_cen,
                                        net->stop_rad, st));
        HIPCHK(launch_prep_splits(net->ns, used, P->n_inst, net->n_relu, P->lo, P->hi, P->bound_of,
                                  P->split_off, P->split_idx, P->split_sign, net->tab, net->infeas,
                                  sp_inst, sp_layer, sp_j, sp_dup, P->n_bounds, sl - 1,
                                  smode == BOUND_STOP_RELU, sl > 0 ? net->stop_cen : nullptr,
                                  sl > 0 ? net->stop_rad : nullptr, st));
        if (inject)
            HIPCHK(launch_beta_sum(nnz, P->rows, P->split_off, P->split_idx, P->split_sign, sp_inst,
                                   sp_layer, sp_dup, P->beta, net->bsum, st));
    } else if (sl > 0) {
        HIPCHK(launch_prep_stop_box(P->n_inst, *SL, net->n_relu, P->lo, P->hi, P->bound_of,
                                    P->n_bounds, smode == BOUND_STOP_RELU, net->stop_cen,
                                    net->stop_rad, st));
    }
    if (conc) {
        HIPCHK(launch_prep_box(P->n_inst, net->C0, net->HW0, P->x_lo, P->x_hi, net->cen, net->rad, st));
    } else {
        HIPCHK(launch_fill(net->cen, (long)P->n_inst * d0, 0.f, st));
        HIPCHK(launch_fill(net->rad, (long)P->n_inst * d0, 0.f, st));
    }
    }

    const long chunk = save ? total : net->max_rows;
    std::vector<long> soff(k + 2, 0);  // offset of saved G_m for m = 1..k
    long lam_off = 0;                  // saved Lambda on z_sl at a linear stop
    std::vector<long> ck(k + 2, -1);   // checkpointed mode: offset of Lambda_t
    int ck_c = 1;
    long seg_off = 0;
    if (save && !recompute) {
        long o = 0;
        for (int m = 1; m <= k; ++m) {
            soff[m] = o;
            o += total * net->d[m - 1];
        }
        lam_off = o;
    } else if (recompute) {
        // G_1 (dense, the concretised layer), then Lambda_t at the checkpoints t = k,
        // k - c, ... >= 2 with c = ceil(sqrt(k - 1)), then the segment area: the largest
        // segment's G (products t .. t - c + 1 keep G on layers t - 1 .. t - c)
        long o = total * net->d[0];
        soff[1] = 0;
        ck_c = 1;
        while ((long)ck_c * ck_c < k - 1) ++ck_c;
        long seg = 0;
        for (int t = k; t >= 2; t -= ck_c) {
            ck[t] = o;
            o += total * net->d[t];
            long s = 0;
            for (int p = t; p >= 2 && p > t - ck_c; --p) s += net->d[p - 1];
            seg = s > seg ? s : seg;
        }
        seg_off = o;
        o += total * seg;
        if (o > net->max_save_rows * (net->d[0] + net->n_relu + net->max_relu_d))
            return fail(BOUND_E_NOMEM, "checkpointed layout exceeds the save workspace");
        const long need = total * net->max_d;
        if (need > net->rbuf_cap) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
                return fail(BOUND_E_NOMEM, "recomputation scratch larger than any earlier pass while "
                                           "the stream is being captured");
            float *r;
            if (!net->alloc(&r, need)) return fail(BOUND_E_NOMEM, "recomputation scratch");
            net->rbuf = r;
            net->rbuf_cap = need;
        }
    }
    for (long img0 = 0; img0 < total; img0 += chunk) {
        const long n_img = total - img0 < chunk ? total - img0 : chunk;
        float *cur = net->buf[0], *nxt = net->buf[1];
        int m_start;
        if (ident) {
            const LayerInfo &li = net->layers[k - 1];
            IdentityParams ip{};
            ip.kind = li.L.kind;
            ip.W = li.L.weight;
            ip.bias_k = li.L.bias;
            ip.ci = li.L.in_c; ip.hi_ = li.L.in_h; ip.wi = li.L.in_w;
            ip.co = li.L.out_c; ip.ho = li.L.out_h; ip.wo = li.L.out_w;
            ip.kh = li.L.kh; ip.kw = li.L.kw; ip.stride = li.L.stride; ip.pad = li.L.pad;
            ip.dk = dk; ip.din = li.din; ip.rpi = rpi; ip.img0 = img0;
            ip.s = net->acc_s; ip.mag = net->acc_mag; ip.low = net->acc_low;
            if (conc_m == k) {
                ip.cen = sl > 0 ? net->stop_cen : net->cen;
                ip.rad = sl > 0 ? net->stop_rad : net->rad;
                ip.emit = conc ? nullptr : out->coeff + img0 * d0;
                ProfScope ps(net, st, "init_identity_conc");
                HIPCHK(launch_init_identity(ip, n_img, true, st));
                m_start = 0;
            } else {
                ip.tab = net->tab + net->relu_off(k - 1);
                ip.tab_ld = net->n_relu;
                ip.bias_m = (smode == BOUND_STOP_LINEAR && sl == k - 1) ? net->zeros : net->bias(k - 1);
                ip.chan_m = net->chan(k - 1);
                ip.out = cur;
                ip.bsum = inject ? net->bsum : nullptr;
                {
                    ProfScope ps(net, st, lbl("init_identity_L%d", k));
                    HIPCHK(launch_init_identity(ip, n_img, false, st));
                }
                m_start = k - 1;
            }
        } else {
            const bound_layer &Lk = net->layers[k - 1].L;
            ProfScope ps(net, st, "init_spec");
            HIPCHK(launch_init_spec(img0, n_img, P->rows, rpi, P->spec, dk, Lk.out_c,
                                    Lk.out_h * Lk.out_w, Lk.bias, cur, net->acc_s, net->acc_mag,
                                    net->acc_low, st));
            m_start = k;
        }
        for (int m = m_start; m >= relax_low; --m) {
            if (recompute && ck[m] >= 0)       // checkpoint: keep Lambda_m for the adjoint
                HIPCHK(hipMemcpyAsync(net->save + ck[m], cur, sizeof(float) * (size_t)(n_img * net->d[m]),
                                      hipMemcpyDeviceToDevice, st));
            RelaxParams rp{};
            rp.out = nxt;
            rp.save = save && !recompute ? net->save + soff[m] : nullptr;
            rp.tab = net->tab + net->relu_off(m - 1);
            rp.tab_ld = net->n_relu;
            // at a linear stop the box is on z_sl itself, so its bias is not added
            rp.bias = (smode == BOUND_STOP_LINEAR && m - 1 == sl) ? net->zeros : net->bias(m - 1);
            rp.chan = net->chan(m - 1);
            rp.D = net->d[m - 1];
            rp.s = net->acc_s;
            rp.mag = net->acc_mag;
            rp.img0 = img0;
            rp.rpi = rpi;
            rp.rrpi = 1.0f / (float)rpi;
            rp.bsum = inject ? net->bsum : nullptr;   // split terms fused into the epilogue
            {
                bound_status bs = det_begin(net, st, m, n_img, rp.det);
                if (bs != BOUND_OK) return bs;
            }
            {
                ProfScope ps(net, st, lbl("bwd_relax_L%d", m));
                const GeomSet &gs = net->layers[m - 1].gT;
                const float *A = cur;
                bound_status bs = run_product(net, st, pkey('R', m), gs, [&](const Plan &pl) {
                    if (rp.det.part) {   // a tuning re-run starts from zeroed slots too
                        const hipError_t e = launch_fill(rp.det.part, n_img * rp.det.nslot * 2, 0.f, st);
                        if (e != hipSuccess) return e;
                    }
                    return gemm_relax(gs, A, n_img, rp, st, pl);
                });
                if (bs != BOUND_OK) return bs;
                if (rp.det.part)
                    HIPCHK(launch_det_reduce(n_img, rp.det.nslot, rp.det.part, rp.s, rp.mag, st));
            }
            {
                bound_status bs = debug_check(net, st, nxt, n_img * net->d[m - 1], lbl("bwd_relax_L%d", m));
                if (bs != BOUND_OK) return bs;
            }
            float *t = cur; cur = nxt; nxt = t;
        }
        if (smode == BOUND_STOP_LINEAR) {
            ProfScope ps(net, st, "stop_conc");
            HIPCHK(launch_box_conc(img0, n_img, rpi, SL->d, cur, net->stop_cen, net->stop_rad,
                                   net->acc_low, net->acc_mag, save ? net->save + lam_off : nullptr, st));
        } else if (m_start >= conc_m) {
            ConcParams cp{};
            const long Dc = net->d[conc_m - 1];
            cp.cen = sl > 0 ? net->stop_cen : net->cen;
            cp.rad = sl > 0 ? net->stop_rad : net->rad;
            cp.D = Dc;
            cp.low = net->acc_low; cp.mag = net->acc_mag;
            cp.save = save ? net->save + soff[conc_m] : nullptr;
            cp.emit = conc ? nullptr : out->coeff + img0 * d0;
            cp.chan = sl > 0 ? SL->C : net->C0;
            cp.hw = sl > 0 ? SL->HW : net->HW0;
            cp.img0 = img0; cp.rpi = rpi; cp.rrpi = 1.0f / (float)rpi;
            bound_status bs = det_begin(net, st, conc_m, n_img, cp.det);
            if (bs != BOUND_OK) return bs;
            {
                ProfScope ps(net, st, lbl("bwd_conc_L%d", conc_m));
                const GeomSet &gs = net->layers[conc_m - 1].gT;
                const float *A = cur;
                bs = run_product(net, st, pkey('C', conc_m), gs, [&](const Plan &pl) {
                    if (cp.det.part) {
                        const hipError_t e = launch_fill(cp.det.part, n_img * cp.det.nslot * 2, 0.f, st);
                        if (e != hipSuccess) return e;
                    }
                    return gemm_conc(gs, A, n_img, cp, st, pl);
                });
                if (bs != BOUND_OK) return bs;
                if (cp.det.part)
                    HIPCHK(launch_det_reduce(n_img, cp.det.nslot, cp.det.part, cp.low, cp.mag, st));
            }
            bs = debug_check(net, st, net->acc_low, n_img, lbl("bwd_conc_L%d", conc_m));
            if (bs != BOUND_OK) return bs;
        }
        ProfScope pf(net, st, "finalize");
        HIPCHK(launch_finalize(img0, n_img, P->rows, rpi, net->acc_s, net->acc_low, net->acc_mag,
                               net->infeas, slack, conc ? out->lower : nullptr,
                               conc ? out->upper : nullptr, ld, conc ? nullptr : out->offset,
                               conc ? nullptr : out->offset_mag, conc ? out->best : nullptr,
                               conc && both ? out->best_upper : nullptr, st));
    }
    if (save) {
        net->saved = true;
        ++net->pass_seq;
        if (out->pass_id) *out->pass_id = net->pass_seq;
        net->s_target = k;
        net->s_rows = rpi;               // rows per instance, the negated spec rows included
        net->s_n_inst = P->n_inst;
        net->s_nnz = used > 0 ? nnz : 0;
        net->s_nnz_arg = nnz;
        net->s_off = soff;
        net->s_stop = sl;
        net->s_mode = smode;
        net->s_lam_off = lam_off;
        net->s_recompute = recompute;
        net->s_inject = inject;
        net->s_c = ck_c;
        net->s_ck = ck;
        net->s_seg_off = seg_off;
        if (net->s_nnz > 0) {
            HIPCHK(hipMemcpyAsync(net->sp_sign, P->split_sign, (size_t)nnz, hipMemcpyDeviceToDevice, st));
        }
    }
    return BOUND_OK;
}

namespace {
// The reverse pass of bound_grad; with as != null the alpha-gradient of each ReLU layer
// goes straight into an Adam step on alpha (bound_grad_adam) instead of grad_alpha.
bound_status grad_impl(bound_net *net, int64_t pass_id, int32_t n_inst, int32_t rows_arg,
                       int32_t nnz, const float *grad_lower, float *grad_alpha,
                       const bound_adam_step *as, float *grad_beta, void *stream, const char *fn) {
    const std::string f(fn);
    if (!net || !grad_lower || (!grad_alpha && !as)) return fail(BOUND_E_ARG, f + ": null argument");
    if (as && (!as->alpha || !as->m || !as->v || as->step < 1))
        return fail(BOUND_E_ARG, f + ": bad alpha step (null buffer or step < 1)");
    if (!net->saved) return fail(BOUND_E_STATE, f + ": no SAVE_FOR_GRAD pass to differentiate");
    if (pass_id != 0 && pass_id != net->pass_seq)
        return fail(BOUND_E_STATE, f + ": pass " + std::to_string(pass_id) +
                                       " is not the last SAVE_FOR_GRAD pass (" +
                                       std::to_string(net->pass_seq) + ") or was invalidated");
    if (n_inst != net->s_n_inst || rows_arg != net->s_rows || (grad_beta && nnz != net->s_nnz_arg))
        return fail(BOUND_E_SHAPE, f + ": n_inst / rows / nnz differ from the saved pass (" +
                                       std::to_string(net->s_n_inst) + " / " +
                                       std::to_string(net->s_rows) + " / " +
                                       std::to_string(net->s_nnz_arg) + ")");
    hipStream_t st = (hipStream_t)stream;
    const int k = net->s_target, rows = net->s_rows;
    const long n_img = (long)net->s_n_inst * rows;
    const long d0 = net->d[0];
    AdamArgs aa{};
    if (as) aa = adam_args(as->step, as->lr, as->b1, as->b2, as->eps, as->grad_scale, as->clip_lo, as->clip_hi);
    {
        ProfScope pz(net, st, "grad_zero");
        if (grad_alpha) HIPCHK(launch_fill(grad_alpha, (long)net->s_n_inst * net->n_relu, 0.f, st));
        if (grad_beta && net->s_nnz > 0) HIPCHK(launch_fill(grad_beta, (long)net->s_nnz * rows, 0.f, st));
    }
    // alpha part of ReLU layer `layer` (0-based) from the row contributions in gcbuf
    auto alpha_part = [&](long D, const LayerShape &S, int layer, long aoff) -> hipError_t {
        if (as)
            return launch_alpha_adam(net->s_n_inst, rows, D, S, layer, net->n_relu, net->srow,
                                     net->slot_count, net->slot_inv, net->slot, net->gcbuf, as->alpha,
                                     as->m, as->v, net->n_relu, aoff, (int)net->s_nnz, net->sp,
                                     net->sp + net->sp_cap, net->sp + 2 * net->sp_cap, aa, st);
        return launch_alpha_grad(net->s_n_inst, rows, D, S, layer, net->n_relu, net->srow,
                                 net->slot_count, net->slot_inv, net->gcbuf, grad_alpha, net->n_relu,
                                 aoff, (int)net->s_nnz, net->sp, net->sp + net->sp_cap,
                                 net->sp + 2 * net->sp_cap, st);
    };
    float *cur = net->buf[0], *nxt = net->buf[1];
    int32_t *sp_inst = net->sp, *sp_layer = net->sp + net->sp_cap, *sp_j = net->sp + 2 * net->sp_cap;
    int32_t *sp_dup = net->sp + 3 * net->sp_cap;
    const int sl = net->s_stop, smode = net->s_mode;
    int m0 = 1;  // first adjoint product
    if (smode == BOUND_STOP_LINEAR) {
        // reverse of the box concretisation of Lambda_sl and of the relaxation of z_sl
        const LayerShape &S = net->ns.l[sl - 1];
        const long Ds = S.d;
        ProfScope pi(net, st, "adj_init");
        HIPCHK(launch_adj_stop_linear(n_img, rows, Ds, net->save + net->s_lam_off,
                                      net->save + net->s_off[sl + 1], net->stop_cen, net->stop_rad,
                                      grad_lower, net->infeas, net->sbar,
                                      net->tab + net->relu_off(sl), net->n_relu,
                                      sl + 1 < k ? cur : nullptr, net->gcbuf, S.C, S.HW, st));
        HIPCHK(alpha_part(Ds, S, sl - 1, net->relu_off(sl)));
        if (grad_beta && net->s_nnz > 0)
            HIPCHK(launch_beta_grad_stop(net->s_nnz, rows, sl - 1, Ds, sp_inst, sp_layer, sp_j,
                                         net->sp_sign, net->save + net->s_lam_off, net->stop_cen,
                                         net->stop_rad, net->sbar, grad_beta, st));
        m0 = sl + 1;
    } else {
        // d lower / d (coefficients at the concretised node) = s_bar (c - sign(.) r)
        const int cm = smode == BOUND_STOP_RELU ? sl + 1 : 1;
        const long Dc = net->d[cm - 1];
        ProfScope pi(net, st, "adj_init");
        HIPCHK(launch_adj_init(n_img, rows, Dc, grad_lower, net->save + net->s_off[cm],
                               sl > 0 ? net->stop_cen : net->cen, sl > 0 ? net->stop_rad : net->rad,
                               net->infeas, cur, net->sbar, st));
        m0 = cm;
    }
    (void)d0;
    // checkpointed mode: G of the products of one segment, recomputed from its checkpoint
    std::vector<const float *> gseg(k + 2, nullptr);
    for (int m = m0; m <= k - 1; ++m) {
        const LayerInfo &li = net->layers[m - 1];
        if (net->s_recompute && gseg[m + 1] == nullptr) {
            // the segment holding product m + 1: checkpoint t >= m + 1, products t .. bot
            int t = m + 1;
            while (t <= k && net->s_ck[t] < 0) ++t;
            const int bot = t - net->s_c + 1 > 2 ? t - net->s_c + 1 : 2;
            const float *A = net->save + net->s_ck[t];
            float *outs[2] = {net->rbuf, nxt};
            long so = net->s_seg_off;       // G of product p: n_img x d_{p-1}, stacked from t down
            for (int p = t; p >= bot; --p) {
                RelaxParams rp{};
                rp.out = outs[(t - p) & 1];
                rp.save = net->save + so;
                so += n_img * net->d[p - 1];
                rp.tab = net->tab + net->relu_off(p - 1);
                rp.tab_ld = net->n_relu;
                rp.bias = net->bias(p - 1);
                rp.chan = net->chan(p - 1);
                rp.D = net->d[p - 1];
                rp.s = net->acc_s;              // scratch here: the pass's sums are final
                rp.mag = net->acc_mag;
                rp.img0 = 0;
                rp.rpi = rows;
                rp.rrpi = 1.0f / (float)rows;
                rp.bsum = net->s_inject ? net->bsum : nullptr;
                {
                    ProfScope ps(net, st, lbl("recompute_L%d", p));
                    const GeomSet &gs = net->layers[p - 1].gT;
                    const float *Ap = A;
                    bound_status bs = run_product(net, st, pkey('R', p), gs, [&](const Plan &pl) {
                        return gemm_relax(gs, Ap, n_img, rp, st, pl);
                    });
                    if (bs != BOUND_OK) return bs;
                }
                gseg[p] = rp.save;
                A = rp.out;
            }
        }
        AdjParams ap{};
        ap.sbar = net->sbar;
        ap.bias = li.L.bias;
        ap.chan = li.L.out_c;
        ap.D = net->d[m];
        ap.gsave = net->s_recompute ? gseg[m + 1] : net->save + net->s_off[m + 1];
        ap.tab = net->tab + net->relu_off(m);
        ap.tab_ld = net->n_relu;
        ap.gout = m + 1 < k ? nxt : nullptr;
        ap.gc = net->gcbuf;
        ap.gbeta = grad_beta && net->s_nnz > 0 ? grad_beta : nullptr;
        ap.hw = li.L.out_h * li.L.out_w;
        ap.rpi = rows;
        ap.rrpi = 1.0f / (float)rows;
        {
            ProfScope ps(net, st, lbl("adj_L%d", m));
            const float *A = cur;
            bound_status bs = run_product(net, st, pkey('A', m), li.gF, [&](const Plan &pl) {
                return gemm_adj(li.gF, A, n_img, ap, st, pl);
            });
            if (bs != BOUND_OK) return bs;
            if (ap.gout) bs = debug_check(net, st, ap.gout, n_img * net->d[m], lbl("adj_L%d", m));
            if (bs != BOUND_OK) return bs;
        }
        {
            ProfScope ps(net, st, as ? "alpha_adam" : "alpha_grad");
            HIPCHK(alpha_part(net->d[m], net->ns.l[m - 1], m - 1, net->relu_off(m)));
        }
        if (grad_beta && net->s_nnz > 0) {
            BetaGradLayer bl{};
            bl.kind = li.L.kind; bl.W = li.L.weight; bl.bias = li.L.bias;
            bl.ci = li.L.in_c; bl.hi_ = li.L.in_h; bl.wi = li.L.in_w;
            bl.co = li.L.out_c; bl.ho = li.L.out_h; bl.wo = li.L.out_w;
            bl.kh = li.L.kh; bl.kw = li.L.kw; bl.stride = li.L.stride; bl.pad = li.L.pad;
            bl.din = li.din; bl.dout = li.dout;
            ProfScope ps(net, st, "beta_grad");
            HIPCHK(launch_beta_grad(net->s_nnz, rows, m - 1, bl, sp_inst, sp_layer, sp_j, sp_dup, net->sp_sign,
                                    cur, net->sbar, net->infeas, grad_beta, st));
        }
        float *t = cur; cur = nxt; nxt = t;
    }
    bound_status bs = as ? debug_check(net, st, as->alpha, (long)net->s_n_inst * net->n_relu, "alpha")
                         : debug_check(net, st, grad_alpha, (long)net->s_n_inst * net->n_relu, "grad_alpha");
    if (bs == BOUND_OK && grad_beta)
        bs = debug_check(net, st, grad_beta, (long)net->s_nnz * rows, "grad_beta");
    return bs;
}
}  // namespace

bound_status bound_grad(bound_net *net, int64_t pass_id, int32_t n_inst, int32_t rows_arg,
                        int32_t nnz, const float *grad_lower, float *grad_alpha, float *grad_beta,
                        void *stream) {
    if (!grad_alpha) return fail(BOUND_E_ARG, "bound_grad: null argument");
    return grad_impl(net, pass_id, n_inst, rows_arg, nnz, grad_lower, grad_alpha, nullptr, grad_beta,
                     stream, "bound_grad");
}

bound_status bound_grad_adam(bound_net *net, int64_t pass_id, int32_t n_inst, int32_t rows_arg,
                             int32_t nnz, const float *grad_lower, const bound_adam_step *alpha_step,
                             float *grad_beta, void *stream) {
    if (!alpha_step) return fail(BOUND_E_ARG, "bound_grad_adam: null argument");
    return grad_impl(net, pass_id, n_inst, rows_arg, nnz, grad_lower, nullptr, alpha_step, grad_beta,
                     stream, "bound_grad_adam");
}

namespace {
bound_status sample_bounds(bound_net *net, int32_t n_sub, int32_t per_sub, const float *x, float *lo,
                           float *hi, float *out, bool merge, void *stream) {
    const char *fn = merge ? "bound_sample_bounds_merge" : "bound_sample_bounds";
    if (!net || n_sub < 1 || per_sub < 1 || !x || (!lo) != (!hi) || (!lo && !out))
        return fail(BOUND_E_ARG, std::string(fn) + ": bad arguments");
    if ((long)per_sub > net->max_rows)
        return fail(BOUND_E_NOMEM, std::string(fn) + ": per_sub > max_rows");
    hipStream_t st = (hipStream_t)stream;
    net->saved = false;
    const int L = net->n_layers;
    const long subs_per_chunk = net->max_rows / per_sub;
    for (long s0 = 0; s0 < n_sub; s0 += subs_per_chunk) {
        const long ns = n_sub - s0 < subs_per_chunk ? n_sub - s0 : subs_per_chunk;
        const long n_img = ns * per_sub;
        float *cur = net->buf[0], *nxt = net->buf[1];
        {
            ProfScope ps(net, st, "fwd_input");
            HIPCHK(launch_to_internal(n_img, net->C0, net->HW0, x + s0 * per_sub * net->d[0], cur, st));
        }
        for (int m = 1; m <= L; ++m) {
            const LayerInfo &li = net->layers[m - 1];
            FwdParams fp{};
            fp.out = nxt;
            fp.bias = li.L.bias;
            fp.D = net->d[m];
            {
                ProfScope ps(net, st, lbl("fwd_L%d", m));
                const float *A = cur;
                bound_status bs = run_product(net, st, pkey('F', m), li.gF, [&](const Plan &pl) {
                    return gemm_fwd(li.gF, A, n_img, fp, st, pl);
                });
                if (bs != BOUND_OK) return bs;
            }
            const bool last = m == L;
            const int C = li.L.out_c, HW = li.L.out_h * li.L.out_w;
            ProfScope pm(net, st, "fwd_minmax");
            if (!last) {
                HIPCHK(launch_sample_minmax(ns, per_sub, net->d[m], C, HW, nxt,
                                            lo ? lo + s0 * net->n_relu + net->relu_off(m) : nullptr,
                                            hi ? hi + s0 * net->n_relu + net->relu_off(m) : nullptr,
                                            net->n_relu, true, nullptr, merge, st));
            } else if (out) {
                HIPCHK(launch_sample_minmax(ns, per_sub, net->d[m], C, HW, nxt, nullptr, nullptr, 0,
                                            false, out + s0 * per_sub * net->d[L], false, st));
            }
            float *t = cur; cur = nxt; nxt = t;
        }
    }
    return BOUND_OK;
}
}  // namespace

bound_status bound_sample_bounds(bound_net *net, int32_t n_sub, int32_t per_sub, const float *x,
                                 float *lo, float *hi, float *out, void *stream) {
    return sample_bounds(net, n_sub, per_sub, x, lo, hi, out, false, stream);
}

bound_status bound_sample_bounds_merge(bound_net *net, int32_t n_sub, int32_t per_sub, const float *x,
                                       float *lo, float *hi, float *out, void *stream) {
    return sample_bounds(net, n_sub, per_sub, x, lo, hi, out, true, stream);
}

bound_status bound_concretize(int32_t n_inst, int32_t rows, int32_t d0, const float *coeff,
                              const float *offset, const float *offset_mag, const float *x_lo,
                              const float *x_hi, int32_t flags, float *lower, void *stream) {
    if (n_inst < 0 || rows < 0 || d0 < 1 || !coeff || !offset || !x_lo || !x_hi || !lower)
        return fail(BOUND_E_ARG, "bound_concretize: bad arguments");
    HIPCHK(launch_concretize(n_inst, rows, d0, coeff, offset, offset_mag, x_lo, x_hi,
                             (flags & BOUND_NO_SLACK) == 0, lower, (hipStream_t)stream));
    return BOUND_OK;
}

bound_status bound_adam(int64_t n, float *param, const float *grad, float *m, float *v, int32_t step,
                        float lr, float b1, float b2, float eps, float grad_scale, float clip_lo,
                        float clip_hi, void *stream) {
    if (n < 0 || (n > 0 && (!param || !grad || !m || !v)) || step < 1)
        return fail(BOUND_E_ARG, "bound_adam: bad arguments");
    HIPCHK(launch_adam(n, param, grad, m, v, step, lr, b1, b2, eps, grad_scale, clip_lo, clip_hi,
                       (hipStream_t)stream));
    return BOUND_OK;
}

bound_status bound_autotune(bound_net *net, const bound_pass *pass, const bound_out *out,
                            const float *grad_lower, void *stream) {
    if (!net || !pass || !out) return fail(BOUND_E_ARG, "bound_autotune: null argument");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(BOUND_E_STATE, "bound_autotune: the stream is being captured");
    const bool grad = grad_lower && (pass->flags & BOUND_SAVE_FOR_GRAD);
    net->tune_report.clear();
    net->tuning = true;
    bound_status s = bound_backward(net, pass, out, stream);
    float *ga = nullptr;
    if (s == BOUND_OK && grad) {
        // the adjoint writes an alpha-gradient; tuning uses a buffer of its own for it
        if (hipMalloc(&ga, sizeof(float) * (size_t)pass->n_inst * (size_t)net->n_relu) != hipSuccess)
            s = fail(BOUND_E_NOMEM, "bound_autotune: gradient scratch");
        else
            s = bound_grad(net, 0, pass->n_inst,
                           pass->rows * ((pass->flags & BOUND_BOTH_SIDES) ? 2 : 1), pass->nnz,
                           grad_lower, ga, nullptr,
                           stream);
    }
    net->tuning = false;
    if (s == BOUND_OK) s = bound_backward(net, pass, out, stream);   // leave valid outputs
    if (ga) {
        hipStreamSynchronize((hipStream_t)stream);
        hipFree(ga);
    }
    return s;
}

int32_t bound_autotune_report(const bound_net *net, char *buf, int32_t cap) {
    if (!net) return -1;
    const int32_t n = (int32_t)net->tune_report.size();
    if (buf && cap > 0) {
        const int32_t m = n < cap - 1 ? n : cap - 1;
        std::memcpy(buf, net->tune_report.data(), (size_t)m);
        buf[m] = 0;
    }
    return n;
}

bound_status bound_set_options(bound_net *net, int32_t options) {
    if (!net || (options & ~(BOUND_OPT_GEMM_ONLY | BOUND_OPT_DIRECT_DMA | BOUND_OPT_CHECK |
                             BOUND_OPT_DETERMINISTIC)))
        return fail(BOUND_E_ARG, "bound_set_options: bad arguments");
    if ((options & BOUND_OPT_DETERMINISTIC) && !net->det_part) {
        long cap = 1;
        for (int m = 1; m <= net->n_layers; ++m)
            cap = std::max(cap, det_slots(net, m));
        float *p = nullptr;
        if (!net->alloc(&p, net->max_rows * cap * 2))
            return fail(BOUND_E_NOMEM, "bound_set_options: deterministic row-sum slots");
        net->det_part = p;
        net->det_cap = cap;
    }
    net->options = options;
    return BOUND_OK;
}

bound_status bound_set_plan(bound_net *net, char product, int32_t layer, int32_t path,
                            int32_t cfg, int32_t cc) {
    if (!net || (product != 'R' && product != 'C' && product != 'A' && product != 'F') ||
        layer < 1 || layer > net->n_layers || path < 0 || path > 2 || cfg < -1 || cfg > 15 ||
        cc < 0 || cc > 1024)
        return fail(BOUND_E_ARG, "bound_set_plan: bad arguments");
    Plan p;
    p.path = path;
    p.cfg = cfg;
    p.cc = cc;
    net->plans[pkey(product, layer)] = p;
    return BOUND_OK;
}

bound_status bound_profile(bound_net *net, int32_t enable) {
    if (!net) return fail(BOUND_E_ARG, "bound_profile: null net");
    net->prof = enable != 0;
    return BOUND_OK;
}

int32_t bound_profile_read(bound_net *net, int32_t cap, char *names, double *total_ms,
                           int32_t *count) {
    if (!net || cap < 0 || (cap > 0 && (!names || !total_ms || !count))) {
        fail(BOUND_E_ARG, "bound_profile_read: bad arguments");
        return BOUND_E_ARG;
    }
    std::map<std::string, std::pair<double, int>> acc;
    std::vector<std::string> order;
    for (auto &r : net->recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            fail(BOUND_E_HIP, "bound_profile_read: event query failed");
            return BOUND_E_HIP;
        }
        if (!acc.count(r.label)) order.push_back(r.label);
        acc[r.label].first += ms;
        acc[r.label].second += 1;
        net->pool.push_back(r.a);
        net->pool.push_back(r.b);
    }
    net->recs.clear();
    int n = 0;
    for (const auto &l : order) {
        if (n >= cap) break;
        std::snprintf(names + 48 * n, 48, "%s", l.c_str());
        total_ms[n] = acc[l].first;
        count[n] = acc[l].second;
        ++n;
    }
    return n;
}

void bound_destroy(bound_net *net) { delete net; }

}  // extern "C"

namespace bp {
// status + message for the other translation units of the library (bab.hip)
bound_status set_error(bound_status s, const std::string &msg) { return fail(s, msg); }
}  // namespace bp
