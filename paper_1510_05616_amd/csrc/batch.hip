// Batched evaluation: many independent channel instances (uneven vesicle and
// node counts) in one persistent launch, captured with the rest of the
// evaluation in a HIP graph.
//
// Work list.  The host cuts every instance's single layer (vesicle sources)
// and double layer (wall sources) into items (instance, op, target tile,
// source split) and sorts each operator's items by estimated cost, longest
// first.  One persistent grid of independent waves per operator pops items
// from that operator's device counter (one vector atomic per item) until its
// list is exhausted; every wave reaches the exit because the counter only
// grows.  Each item writes its own
// FP64 partial slot, and a final per-target pass adds the slots in fixed
// order, so the result is bitwise deterministic whatever order the items ran
// in.  Uneven vesicle sizes are absorbed because items tile over nodes, not
// over curves.
//
// Graph.  Upload of the descriptor tables (from a pinned host buffer),
// counter reset (a kernel, not a memset), source preparation, Kress tables,
// own-curve sums, the persistent pair kernel and the final pass are captured
// once per argument set; later calls with the same arguments are one
// hipGraphLaunch on the caller's stream.
//
// Autotuning.  On the first call for a size bucket the host times a small
// grid of tile shapes (targets per lane, superblocks per split, waves per
// CU) with HIP events on the real inputs and keeps the fastest; the choice
// is cached per (architecture, precision, size bucket) in memory and in a
// JSON file.
#include "pair_impl.h"
#include "prep_impl.h"
#include "self_impl.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>

namespace s2d {

struct BatchInst {
    PairArgs pa[2];          // [0] single layer from vesicles, [1] double layer from walls
    s2d_curves src[2];
    s2d_targets trg[2];
    double mu;
    double *u, *v;
    double *self;            // [2][n_trg] own-curve Kress sums, or NULL
    double *kress;           // [n_src ves] Kress table, or NULL
};

struct BatchItem {
    int32_t inst, op, tile, split;
};

struct BatchTables {
    const BatchInst *inst;
    const BatchItem *items;                        // single-layer items, then double-layer items
    int64_t n_items;
    int64_t n_items_op[2];                         // items per op
    unsigned long long *counter;                   // [2]: next item per op
    const int64_t *src_pad_off0, *src_pad_off1;   // prefix sums of padded sources per op
    const int64_t *sb_off;                         // prefix sums of single-layer superblocks
    const int64_t *curve_pre;                      // prefix sums of vesicle curve counts
    const int64_t *trg_off;                        // prefix sums of target counts
    int32_t n_inst;
};

// largest k in [0, n) with off[k] <= g (off ascending, off[0] = 0)
__device__ __forceinline__ int find_inst(const int64_t *__restrict__ off, int n, int64_t g) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void batch_reset(unsigned long long *counter) {
    if (threadIdx.x < 2 && blockIdx.x == 0) counter[threadIdx.x] = 0ull;
}

// FP64: one thread per padded source; FP32C: one thread per sub-block
// (the prefix sums count padded sources; sub-blocks never straddle instances).
template <int PREC>
__global__ __launch_bounds__(256) void batch_prep(BatchTables t, int op) {
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t g = PREC == S2D_FP64 ? g0 : g0 * kSubBlock;
    const int64_t *off = op == 0 ? t.src_pad_off0 : t.src_pad_off1;
    if (g >= off[t.n_inst]) return;
    const int k = find_inst(off, t.n_inst, g);
    const BatchInst &I = t.inst[k];
    const int64_t j = g - off[k];
    const s2d_curves &s = I.src[op];
    void *rec = (void *)I.pa[op].rec;
    if (PREC == S2D_FP64) {
        if (op == 0) prep_one64<S2D_OP_SLP>(j, s.n_nodes, s.x, s.y, s.nx, s.ny, s.w, s.fx, s.fy, rec);
        else prep_one64<S2D_OP_DLP>(j, s.n_nodes, s.x, s.y, s.nx, s.ny, s.w, s.fx, s.fy, rec);
    } else {
        SubInfo *sub = (SubInfo *)I.pa[op].sub;
        if (op == 0)
            prep_sub32<S2D_OP_SLP>(j / kSubBlock, s.n_nodes, s.x, s.y, s.nx, s.ny, s.w, s.fx, s.fy, rec, sub);
        else
            prep_sub32<S2D_OP_DLP>(j / kSubBlock, s.n_nodes, s.x, s.y, s.nx, s.ny, s.w, s.fx, s.fy, rec, sub);
    }
}

__global__ __launch_bounds__(256) void batch_sbsum(BatchTables t) {
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;    // a wave per superblock
    if (g >= t.sb_off[t.n_inst]) return;                                          // wave-uniform
    const int k = find_inst(t.sb_off, t.n_inst, g);
    const BatchInst &I = t.inst[k];
    const s2d_curves &s = I.src[0];
    sbsum_wave(g - t.sb_off[k], s.n_nodes, s.w, s.fx, s.fy, (double *)I.pa[0].sbsum, threadIdx.x & (kWave - 1));
}

__global__ __launch_bounds__(256) void batch_kress_table(BatchTables t) {
    __shared__ double ctab[kCosTab];
    const int64_t g = blockIdx.x;
    if (g >= t.curve_pre[t.n_inst]) return;
    const int k = find_inst(t.curve_pre, t.n_inst, g);
    const BatchInst &I = t.inst[k];
    if (!I.kress) return;                                     // block-uniform
    kress_table_curve(I.src[0].curve_off, (int32_t)(g - t.curve_pre[k]), I.src[0].n_nodes, I.kress, ctab);
}

__global__ __launch_bounds__(256) void batch_kress_self(BatchTables t) {
    __shared__ __attribute__((aligned(16))) double ltab[kLogTabWords];
    fill_log_table(ltab);                           // before any thread returns
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= t.trg_off[t.n_inst]) return;
    const int k = find_inst(t.trg_off, t.n_inst, g);
    const BatchInst &I = t.inst[k];
    if (!I.self) return;
    const int64_t i = g - t.trg_off[k];
    const s2d_curves &s = I.src[0];
    double sx, sy;
    kress_self_one(i, s.n_nodes, I.trg[0].on_curve, I.trg[0].on_node, s.curve_off, s.n_curves, s.x, s.y, s.nx,
                   s.ny, s.w, s.fx, s.fy, I.kress, ltab, sx, sy);
    I.self[i] = sx;
    I.self[I.trg[0].n + i] = sy;
}

// One persistent grid per operator, so that each body gets its own register
// allocation (the single layer needs about twice the registers of the double
// layer); each drains its own contiguous range of the work list.
template <int OP, int PREC, int TPT>
__global__ __launch_bounds__(kBlock) void batch_pair(BatchTables t) {
    __shared__ __attribute__((aligned(16))) double ltab[kLogTabWords];
    if (PREC == S2D_FP64 && OP == S2D_OP_SLP) fill_log_table(ltab);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t first = OP == S2D_OP_SLP ? 0 : t.n_items_op[0];
    const int64_t count = t.n_items_op[OP];
    for (;;) {
        int it = 0;
        if (lane == 0) it = (int)atomicAdd(t.counter + OP, 1ull);
        const int64_t k = __builtin_amdgcn_readfirstlane(it);      // lane 0's value, wave-uniform
        if (k >= count) break;                                     // every wave gets here
        // the tables were uploaded before the launch: read them as invariant
        const BatchItem w = load_ro<BatchItem>(t.items, first + k);
        const PairArgs a = load_ro<PairArgs>(&t.inst[w.inst].pa[OP], 0);
        pair_tile<OP, PREC, TPT, 3>(a, w.tile, w.split, lane, ltab);    // images -1, 0, 1
    }
}

__global__ __launch_bounds__(256) void batch_final(BatchTables t) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= t.trg_off[t.n_inst]) return;
    const int k = find_inst(t.trg_off, t.n_inst, g);
    const BatchInst &I = t.inst[k];
    const int64_t i = g - t.trg_off[k];
    const int64_t n = I.trg[0].n;
    double sx = 0.0, sy = 0.0, dx = 0.0, dy = 0.0;
    for (int s = 0; s < I.pa[0].n_splits; ++s) {
        sx += I.pa[0].part[(int64_t)(2 * s) * n + i];
        sy += I.pa[0].part[(int64_t)(2 * s + 1) * n + i];
    }
    if (I.self) {
        sx += I.self[i];
        sy += I.self[n + i];
    }
    for (int s = 0; s < I.pa[1].n_splits; ++s) {
        dx += I.pa[1].part[(int64_t)(2 * s) * n + i];
        dy += I.pa[1].part[(int64_t)(2 * s + 1) * n + i];
    }
    const s2d_curves &w = I.src[1];
    if (I.trg[1].on_curve)
        dlp_diag_one(i, w.n_nodes, I.trg[1].on_curve, I.trg[1].on_node, w.curve_off, w.n_curves, w.nx, w.ny, w.w,
                     w.kappa, w.fx, w.fy, dx, dy);
    const double ps = 1.0 / (4.0 * M_PI * I.mu), pd = 1.0 / M_PI;
    I.u[i] = ps * sx + pd * dx;
    I.v[i] = ps * sy + pd * dy;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

struct TuneChoice {
    int tpt, sbps, wpc;
    double ms;
};

std::mutex g_bmu;
std::map<std::string, TuneChoice> g_tune;
bool g_tune_loaded = false;

std::string tune_path() {
    const char *p = std::getenv("S2D_TUNE_CACHE");
    if (p && *p) return p;
    const char *h = std::getenv("HOME");
    return std::string(h && *h ? h : "/tmp") + "/.cache/stokes2d_tune.json";
}

// The file is a flat JSON object {"key": [tpt, sbps, wpc, ms], ...}.
void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    FILE *f = std::fopen(tune_path().c_str(), "r");
    if (!f) return;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = txt.find('"', pos)) != std::string::npos) {
        const size_t e = txt.find('"', pos + 1);
        if (e == std::string::npos) break;
        const std::string key = txt.substr(pos + 1, e - pos - 1);
        const size_t lb = txt.find('[', e), rb = txt.find(']', e);
        if (lb == std::string::npos || rb == std::string::npos) break;
        TuneChoice c{};
        if (std::sscanf(txt.c_str() + lb + 1, "%d , %d , %d , %lf", &c.tpt, &c.sbps, &c.wpc, &c.ms) == 4 &&
            (c.tpt == 1 || c.tpt == 2 || c.tpt == 4) && c.sbps > 0 && c.wpc > 0)
            g_tune[key] = c;
        pos = rb + 1;
    }
}

void tune_save() {
    const std::string path = tune_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash);
        // create the directory if needed (best effort)
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') {
                const std::string sub = dir.substr(0, i);
                (void)mkdir(sub.c_str(), 0755);
            }
    }
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (auto &kv : g_tune)
        std::fprintf(f, "  \"%s\": [%d, %d, %d, %.6f]%s\n", kv.first.c_str(), kv.second.tpt, kv.second.sbps,
                     kv.second.wpc, kv.second.ms, ++i < g_tune.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path.c_str());
}

struct Layout {
    size_t off_inst, off_items, off_pre, off_counter, off_data, total;
    int64_t n_items;
};

struct BatchPlan {
    std::vector<uint64_t> key;
    int device = 0, mode = 0;
    TuneChoice cfg{};
    Layout lay{};
    void *ws = nullptr;
    void *host = nullptr;         // pinned table image
    size_t host_bytes = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchPlan() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (cap) hipStreamDestroy(cap);
        if (host) hipHostFree(host);
    }
};

std::vector<std::unique_ptr<BatchPlan>> g_plans;
constexpr size_t kMaxPlans = 16;

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t recb(int op, int mode) {
    if (op == 0) return mode == S2D_FP64 ? sizeof(RecSlp64) : sizeof(RecSlp32);
    return mode == S2D_FP64 ? sizeof(RecDlp64) : sizeof(RecDlp32);
}

// Per-instance sizes for a tile configuration.
struct InstGeom {
    int64_t n_sb[2], n_tiles, n_splits[2], sbps;
    size_t off_rec[2], off_sub[2], off_sbsum, off_part[2], off_self, off_kress, bytes;
    bool self;
};

InstGeom inst_geom(const s2d_instance &I, int mode, const TuneChoice &c) {
    InstGeom g{};
    const s2d_curves *src[2] = {&I.ves, &I.wall};
    const int64_t n = I.trg_ves.n;
    g.n_tiles = (n + (int64_t)kWave * c.tpt - 1) / ((int64_t)kWave * c.tpt);
    g.sbps = c.sbps;
    size_t off = 0;
    for (int op = 0; op < 2; ++op) {
        g.n_sb[op] = (src[op]->n_nodes + kSuperBlock - 1) / kSuperBlock;
        g.n_splits[op] = n > 0 ? (g.n_sb[op] + c.sbps - 1) / c.sbps : 0;
        g.off_rec[op] = off;
        off = al256(off + (size_t)g.n_sb[op] * kSuperBlock * recb(op, mode));
        g.off_sub[op] = off;
        if (mode == S2D_FP32C) off = al256(off + (size_t)g.n_sb[op] * (kSuperBlock / kSubBlock) * sizeof(SubInfo));
    }
    g.off_sbsum = off;
    if (mode == S2D_FP32C) off = al256(off + (size_t)g.n_sb[0] * 16);
    for (int op = 0; op < 2; ++op) {
        g.off_part[op] = off;
        off = al256(off + (size_t)g.n_splits[op] * 2 * (size_t)n * 8);
    }
    g.self = I.trg_ves.on_curve != nullptr && n > 0;
    g.off_self = off;
    g.off_kress = off;
    if (g.self) {
        off = al256(off + 2 * (size_t)n * 8);
        g.off_kress = off;
        off = al256(off + (size_t)I.ves.n_nodes * 8);
    }
    g.bytes = off;
    return g;
}

Layout layout(int32_t n_inst, const s2d_instance *inst, int mode, const TuneChoice &c,
              std::vector<InstGeom> *geoms) {
    Layout L{};
    int64_t n_items = 0;
    size_t data = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        InstGeom g = inst_geom(inst[k], mode, c);
        n_items += g.n_tiles * (g.n_splits[0] + g.n_splits[1]);
        data += g.bytes;
        if (geoms) geoms->push_back(g);
    }
    L.n_items = n_items;
    L.off_inst = 0;
    L.off_items = al256(sizeof(BatchInst) * (size_t)n_inst);
    L.off_pre = al256(L.off_items + sizeof(BatchItem) * (size_t)n_items);
    L.off_counter = al256(L.off_pre + sizeof(int64_t) * 5 * ((size_t)n_inst + 1));
    L.off_data = al256(L.off_counter + 16);
    L.total = L.off_data + data;
    return L;
}

const TuneChoice kCandidates64[] = {{1, 2, 16, 0}, {1, 4, 16, 0}, {1, 8, 16, 0}, {2, 4, 16, 0}, {1, 4, 24, 0}};
const TuneChoice kCandidates32[] = {{1, 2, 24, 0}, {1, 4, 24, 0}, {1, 8, 24, 0}, {1, 4, 32, 0},
                                    {2, 4, 16, 0}, {2, 4, 24, 0}, {2, 8, 24, 0}, {2, 4, 32, 0},
                                    {2, 8, 32, 0}};

void candidates(int mode, std::vector<TuneChoice> &out) {
    out.clear();
    if (mode == S2D_FP64)
        out.assign(std::begin(kCandidates64), std::end(kCandidates64));
    else
        out.assign(std::begin(kCandidates32), std::end(kCandidates32));
}

TuneChoice default_choice(int mode) { return mode == S2D_FP64 ? TuneChoice{1, 4, 16, 0} : TuneChoice{1, 4, 24, 0}; }

std::string bucket_key(int mode, int32_t n_inst, const s2d_instance *inst) {
    double pairs = 0;
    for (int32_t k = 0; k < n_inst; ++k)
        pairs += (double)inst[k].trg_ves.n * (double)(inst[k].ves.n_nodes + inst[k].wall.n_nodes) * 3.0;
    const int b = pairs > 0 ? (int)std::floor(std::log2(pairs)) : 0;
    return std::string("gfx950/batch/") + (mode == S2D_FP64 ? "fp64" : "fp32c") + "/2^" + std::to_string(b);
}

template <int PREC, int TPT>
hipError_t launch_batch_pair(const BatchTables &t, int blocks, hipStream_t st) {
    if (t.n_items_op[0] > 0)
        hipLaunchKernelGGL((batch_pair<S2D_OP_SLP, PREC, TPT>), dim3(blocks), dim3(kBlock), 0, st, t);
    if (t.n_items_op[1] > 0)
        hipLaunchKernelGGL((batch_pair<S2D_OP_DLP, PREC, TPT>), dim3(blocks), dim3(kBlock), 0, st, t);
    return hipGetLastError();
}

hipError_t record_graph(BatchPlan &P, const BatchTables &t, int n_pre_targets, int64_t tot_src0, int64_t tot_src1,
                        int64_t tot_sb, int64_t tot_curves, int64_t tot_trg, bool any_self, int cus) {
    hipStream_t st = P.cap;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    (void)n_pre_targets;
    auto done = [&](hipError_t err) {
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(st, &g);
        if (err == hipSuccess) err = e2;
        if (err != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return err;
        }
        P.graph = g;
        return hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0);
    };
    e = hipMemcpyAsync(P.ws, P.host, P.host_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return done(e);
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(64), 0, st, t.counter);
    const int prec = P.mode;
    for (int op = 0; op < 2; ++op) {
        const int64_t tot = op == 0 ? tot_src0 : tot_src1;
        if (tot <= 0) continue;
        if (prec == S2D_FP64)
            hipLaunchKernelGGL(batch_prep<S2D_FP64>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, t, op);
        else
            hipLaunchKernelGGL(batch_prep<S2D_FP32C>, dim3((unsigned)((tot / kSubBlock + 255) / 256)), dim3(256), 0,
                               st, t, op);
    }
    if (prec == S2D_FP32C && tot_sb > 0)
        hipLaunchKernelGGL(batch_sbsum, dim3((unsigned)((tot_sb + 3) / 4)), dim3(256), 0, st, t);
    if (any_self && tot_curves > 0) {
        hipLaunchKernelGGL(batch_kress_table, dim3((unsigned)tot_curves), dim3(256), 0, st, t);
        hipLaunchKernelGGL(batch_kress_self, dim3((unsigned)((tot_trg + 255) / 256)), dim3(256), 0, st, t);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return done(e);
    if (t.n_items > 0) {
        const int blocks = std::max(1, cus * P.cfg.wpc / kWavesPerBlock);
        const int tpt = P.cfg.tpt;
        if (prec == S2D_FP64) {
            e = tpt == 1 ? launch_batch_pair<S2D_FP64, 1>(t, blocks, st)
                : tpt == 2 ? launch_batch_pair<S2D_FP64, 2>(t, blocks, st) : launch_batch_pair<S2D_FP64, 4>(t, blocks, st);
        } else {
            e = tpt == 1 ? launch_batch_pair<S2D_FP32C, 1>(t, blocks, st)
                : tpt == 2 ? launch_batch_pair<S2D_FP32C, 2>(t, blocks, st) : launch_batch_pair<S2D_FP32C, 4>(t, blocks, st);
        }
        if (e != hipSuccess) return done(e);
    }
    if (tot_trg > 0) hipLaunchKernelGGL(batch_final, dim3((unsigned)((tot_trg + 255) / 256)), dim3(256), 0, st, t);
    return done(hipGetLastError());
}

// Builds the table image, the work list and the graph for one configuration.
int build_plan(BatchPlan &P, int mode, int32_t n_inst, const s2d_instance *inst, void *ws, size_t ws_bytes,
               const TuneChoice &c, int cus, std::string &err) {
    P.mode = mode;
    P.cfg = c;
    P.ws = ws;
    std::vector<InstGeom> geoms;
    P.lay = layout(n_inst, inst, mode, c, &geoms);
    if (ws_bytes < P.lay.total) {
        err = "batch workspace too small: need " + std::to_string(P.lay.total) + " bytes";
        return S2D_EWORKSPACE;
    }
    const Layout &L = P.lay;
    P.host_bytes = L.off_counter;       // tables only; the counter is reset by a kernel
    if (hipHostMalloc(&P.host, std::max<size_t>(P.host_bytes, 256), hipHostMallocDefault) != hipSuccess) {
        err = "hipHostMalloc failed";
        return S2D_EHIP;
    }
    std::memset(P.host, 0, P.host_bytes);
    char *hb = (char *)P.host;
    char *db = (char *)ws;
    BatchInst *bi = (BatchInst *)(hb + L.off_inst);
    BatchItem *items = (BatchItem *)(hb + L.off_items);
    int64_t *pre = (int64_t *)(hb + L.off_pre);
    const size_t np = (size_t)n_inst + 1;
    int64_t *p_src0 = pre, *p_src1 = pre + np, *p_sb = pre + 2 * np, *p_cur = pre + 3 * np, *p_trg = pre + 4 * np;
    p_src0[0] = p_src1[0] = p_sb[0] = p_cur[0] = p_trg[0] = 0;
    size_t data = L.off_data;
    bool any_self = false;
    struct Cost {
        double cost;
        BatchItem it;
    };
    std::vector<Cost> work;
    work.reserve((size_t)L.n_items);
    const double wslp = mode == S2D_FP64 ? 2.7 : 1.2;
    for (int32_t k = 0; k < n_inst; ++k) {
        const s2d_instance &I = inst[k];
        const InstGeom &g = geoms[k];
        BatchInst &B = bi[k];
        B.src[0] = I.ves;
        B.src[1] = I.wall;
        B.trg[0] = I.trg_ves;
        B.trg[1] = I.trg_wall;
        B.mu = I.mu;
        B.u = I.u;
        B.v = I.v;
        B.self = g.self ? (double *)(db + data + g.off_self) : nullptr;
        B.kress = g.self ? (double *)(db + data + g.off_kress) : nullptr;
        any_self |= g.self;
        const int64_t n = I.trg_ves.n;
        for (int op = 0; op < 2; ++op) {
            PairArgs &a = B.pa[op];
            const s2d_curves &s = op == 0 ? I.ves : I.wall;
            const s2d_targets &tr = op == 0 ? I.trg_ves : I.trg_wall;
            a.rec = db + data + g.off_rec[op];
            a.sbsum = (op == 0 && mode == S2D_FP32C) ? (const double *)(db + data + g.off_sbsum) : nullptr;
            a.sub = mode == S2D_FP32C ? (const SubInfo *)(db + data + g.off_sub[op]) : nullptr;
            a.n_src = s.n_nodes;
            a.tx = tr.x;
            a.ty = tr.y;
            a.on_curve = tr.on_curve;
            a.on_node = tr.on_node;
            a.curve_off = s.curve_off;
            a.n_curves = s.n_curves;
            a.n_trg = n;
            a.n_tiles = g.n_tiles;
            a.n_splits = (int32_t)g.n_splits[op];
            a.sb_per_split = g.sbps;
            a.n_sb = g.n_sb[op];
            a.d = I.d;
            a.img_lo = -1;
            a.img_hi = 1;
            a.part = (double *)(db + data + g.off_part[op]);
            for (int64_t tl = 0; tl < g.n_tiles; ++tl) {
                const int64_t act = std::min<int64_t>((int64_t)kWave * c.tpt, n - tl * kWave * c.tpt);
                for (int64_t sp = 0; sp < g.n_splits[op]; ++sp) {
                    const int64_t sb0 = sp * g.sbps, sb1 = std::min<int64_t>(sb0 + g.sbps, g.n_sb[op]);
                    const double nsrc = (double)std::min<int64_t>(sb1 * kSuperBlock, s.n_nodes) - sb0 * kSuperBlock;
                    // a wave pays for all its lanes: cost in wave-pairs
                    const double lanes = (double)kWave * c.tpt;
                    (void)act;
                    work.push_back({lanes * nsrc * 3.0 * (op == 0 ? wslp : 1.0),
                                    BatchItem{k, op, (int32_t)tl, (int32_t)sp}});
                }
            }
        }
        p_src0[k + 1] = p_src0[k] + g.n_sb[0] * kSuperBlock;
        p_src1[k + 1] = p_src1[k] + g.n_sb[1] * kSuperBlock;
        p_sb[k + 1] = p_sb[k] + g.n_sb[0];
        p_cur[k + 1] = p_cur[k] + I.ves.n_curves;
        p_trg[k + 1] = p_trg[k] + n;
        data += g.bytes;
    }
    // per op, longest first
    std::stable_sort(work.begin(), work.end(), [](const Cost &a, const Cost &b) {
        return a.it.op != b.it.op ? a.it.op < b.it.op : a.cost > b.cost;
    });
    int64_t n_op[2] = {0, 0};
    for (size_t i = 0; i < work.size(); ++i) {
        items[i] = work[i].it;
        ++n_op[work[i].it.op];
    }

    BatchTables t{};
    t.inst = (const BatchInst *)(db + L.off_inst);
    t.items = (const BatchItem *)(db + L.off_items);
    t.n_items = (int64_t)work.size();
    t.n_items_op[0] = n_op[0];
    t.n_items_op[1] = n_op[1];
    t.counter = (unsigned long long *)(db + L.off_counter);
    const int64_t *dpre = (const int64_t *)(db + L.off_pre);
    t.src_pad_off0 = dpre;
    t.src_pad_off1 = dpre + np;
    t.sb_off = dpre + 2 * np;
    t.curve_pre = dpre + 3 * np;
    t.trg_off = dpre + 4 * np;
    t.n_inst = n_inst;
    if (hipStreamCreateWithFlags(&P.cap, hipStreamNonBlocking) != hipSuccess) {
        err = "hipStreamCreate failed";
        return S2D_EHIP;
    }
    hipError_t e = record_graph(P, t, 0, p_src0[n_inst], p_src1[n_inst], p_sb[n_inst], p_cur[n_inst],
                                p_trg[n_inst], any_self, cus);
    if (e != hipSuccess) {
        err = std::string("batch graph capture: ") + hipGetErrorString(e);
        return S2D_EHIP;
    }
    return S2D_OK;
}

void push_key(std::vector<uint64_t> &k, const void *p) { k.push_back((uint64_t)(uintptr_t)p); }
void push_key(std::vector<uint64_t> &k, double d) {
    uint64_t u;
    std::memcpy(&u, &d, 8);
    k.push_back(u);
}

std::vector<uint64_t> make_key(int dev, int mode, int32_t n_inst, const s2d_instance *inst, void *ws,
                               size_t ws_bytes) {
    std::vector<uint64_t> k;
    k.reserve(8 + (size_t)n_inst * 40);
    k.push_back((uint64_t)dev);
    k.push_back((uint64_t)mode);
    k.push_back((uint64_t)n_inst);
    push_key(k, ws);
    k.push_back((uint64_t)ws_bytes);
    for (int32_t i = 0; i < n_inst; ++i) {
        const s2d_instance &I = inst[i];
        for (const s2d_curves *c : {&I.ves, &I.wall}) {
            k.push_back((uint64_t)c->n_nodes);
            k.push_back((uint64_t)c->n_curves);
            for (const void *p : {(const void *)c->curve_off, (const void *)c->x, (const void *)c->y,
                                  (const void *)c->nx, (const void *)c->ny, (const void *)c->w,
                                  (const void *)c->kappa, (const void *)c->fx, (const void *)c->fy})
                push_key(k, p);
        }
        for (const s2d_targets *t : {&I.trg_ves, &I.trg_wall}) {
            k.push_back((uint64_t)t->n);
            for (const void *p : {(const void *)t->x, (const void *)t->y, (const void *)t->on_curve,
                                  (const void *)t->on_node})
                push_key(k, p);
        }
        push_key(k, I.d);
        push_key(k, I.mu);
        push_key(k, (const void *)I.u);
        push_key(k, (const void *)I.v);
    }
    return k;
}

}  // namespace

// Entry points called from api.hip (argument checks done there).
size_t batch_workspace_size(int mode, int32_t n_inst, const s2d_instance *inst) {
    std::vector<TuneChoice> cands;
    candidates(mode, cands);
    size_t mx = 0;
    for (auto &c : cands) mx = std::max(mx, layout(n_inst, inst, mode, c, nullptr).total);
    return mx;
}

int batch_eval(int dev, int cus, int mode, int32_t n_inst, const s2d_instance *inst, void *ws, size_t ws_bytes,
               hipStream_t stream, std::string &err) {
    std::vector<uint64_t> key = make_key(dev, mode, n_inst, inst, ws, ws_bytes);
    std::lock_guard<std::mutex> lk(g_bmu);
    for (auto &p : g_plans) {
        if (p->key == key) {
            hipError_t e = hipGraphLaunch(p->exec, stream);
            if (e != hipSuccess) {
                err = std::string("hipGraphLaunch: ") + hipGetErrorString(e);
                return S2D_EHIP;
            }
            return S2D_OK;
        }
    }
    // the plan's kernels read caller data that earlier work on `stream` may produce
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
        return S2D_EHIP;
    }
    tune_load();
    const std::string bk = bucket_key(mode, n_inst, inst);
    TuneChoice choice = default_choice(mode);
    std::unique_ptr<BatchPlan> best;
    auto it = g_tune.find(bk);
    const char *tune_env = std::getenv("S2D_TUNE");
    const bool tune = !(tune_env && tune_env[0] == '0');
    if (it != g_tune.end()) {
        choice = it->second;
    } else if (tune) {
        std::vector<TuneChoice> cands;
        candidates(mode, cands);
        hipEvent_t a, b;
        hipEventCreate(&a);
        hipEventCreate(&b);
        double best_ms = 1e300;
        for (auto &c : cands) {
            auto P = std::make_unique<BatchPlan>();
            int rc = build_plan(*P, mode, n_inst, inst, ws, ws_bytes, c, cus, err);
            if (rc != S2D_OK) {
                hipEventDestroy(a);
                hipEventDestroy(b);
                return rc;
            }
            hipGraphLaunch(P->exec, P->cap);                 // warm-up
            hipEventRecord(a, P->cap);
            for (int r = 0; r < 2; ++r) hipGraphLaunch(P->exec, P->cap);
            hipEventRecord(b, P->cap);
            e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e != hipSuccess) {
                hipEventDestroy(a);
                hipEventDestroy(b);
                err = std::string("batch tuning: ") + hipGetErrorString(e);
                return S2D_EHIP;
            }
            if (ms / 2 < best_ms) {
                best_ms = ms / 2;
                choice = c;
                choice.ms = best_ms;
                best = std::move(P);
            }
        }
        hipEventDestroy(a);
        hipEventDestroy(b);
        g_tune[bk] = choice;
        tune_save();
    }
    if (!best) {
        best = std::make_unique<BatchPlan>();
        int rc = build_plan(*best, mode, n_inst, inst, ws, ws_bytes, choice, cus, err);
        if (rc != S2D_OK) return rc;
    }
    best->key = std::move(key);
    best->device = dev;
    e = hipGraphLaunch(best->exec, stream);
    if (e != hipSuccess) {
        err = std::string("hipGraphLaunch: ") + hipGetErrorString(e);
        return S2D_EHIP;
    }
    if (g_plans.size() >= kMaxPlans) {
        hipStreamSynchronize(stream);
        g_plans.erase(g_plans.begin());
    }
    g_plans.push_back(std::move(best));
    return S2D_OK;
}

int batch_release() {
    std::lock_guard<std::mutex> lk(g_bmu);
    hipDeviceSynchronize();
    g_plans.clear();
    return S2D_OK;
}

int batch_tuned(int mode, int32_t n_inst, const s2d_instance *inst, int *tpt, int *sbps, int *wpc) {
    std::lock_guard<std::mutex> lk(g_bmu);
    tune_load();
    auto it = g_tune.find(bucket_key(mode, n_inst, inst));
    TuneChoice c = it != g_tune.end() ? it->second : default_choice(mode);
    *tpt = c.tpt;
    *sbps = c.sbps;
    *wpc = c.wpc;
    return it != g_tune.end() ? 1 : 0;
}

}  // namespace s2d
