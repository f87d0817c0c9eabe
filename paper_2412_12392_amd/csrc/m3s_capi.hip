// C ABI of libm3s (declared in include/m3s.h): host-side validation, workspace
// layout, dispatch, hipGraph capture/replay and the batched-launch autotuner.
// Host code only; the kernels live in m3s_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "m3s.h"
#include "m3s_internal.h"

using m3s::EdgeArgs;

namespace {

thread_local std::string g_last_error;
thread_local int32_t g_last_grid = 0, g_last_tile = 0, g_last_margin = 0, g_last_unroll = 0;

m3s_status fail(m3s_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

m3s_status hip_fail(hipError_t e, const char* what) {
    return fail(M3S_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// ---------------------------------------------------------------- device info

struct DeviceInfo {
    bool checked = false;
    bool supported = false;
    int cus = 0;
    std::string arch;
};
std::mutex g_dev_mu;
std::map<int, DeviceInfo> g_devices;

m3s_status current_device(int* dev, DeviceInfo* info) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceInfo& d = g_devices[*dev];
    if (!d.checked) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, *dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        d.arch = prop.gcnArchName;
        d.supported = d.arch.compare(0, 6, "gfx950") == 0;
        d.cus = prop.multiProcessorCount;
        d.checked = true;
    }
    *info = d;
    if (!d.supported) return fail(M3S_ERR_UNSUPPORTED, "device %d is %s; libm3s is built for gfx950 only", *dev, d.arch.c_str());
    return M3S_OK;
}

// ---------------------------------------------------------------- validation

m3s_status check_params(const m3s_params* P) {
    if (P->max_iter < 0 || P->max_iter > M3S_MAX_ITER) return fail(M3S_ERR_PARAM, "max_iter %d outside [0, %d]", P->max_iter, M3S_MAX_ITER);
    if (!(std::isfinite(P->lambda_init) && P->lambda_init > 0.f)) return fail(M3S_ERR_PARAM, "lambda_init must be finite and > 0");
    if (P->refine_radius < 0 || P->refine_radius > M3S_MAX_RADIUS)
        return fail(M3S_ERR_PARAM, "refine_radius %d outside [0, %d]", P->refine_radius, M3S_MAX_RADIUS);
    if (P->refine_levels < 1 || P->refine_levels > M3S_MAX_LEVELS)
        return fail(M3S_ERR_PARAM, "refine_levels %d outside [1, %d]", P->refine_levels, M3S_MAX_LEVELS);
    if (!std::isfinite(P->conf_min)) return fail(M3S_ERR_PARAM, "conf_min must be finite");
    if (std::isnan(P->max_theta) || P->max_theta < 0.f) return fail(M3S_ERR_PARAM, "max_theta must be >= 0");
    if (std::isnan(P->max_dist) || !(P->max_dist > 0.f)) return fail(M3S_ERR_PARAM, "max_dist must be > 0 (inf disables)");
    return M3S_OK;
}

m3s_status check_shape(int32_t H, int32_t W) {
    if (H < 2 || W < 2) return fail(M3S_ERR_SHAPE, "H and W must be >= 2 (got %d x %d)", H, W);
    if ((int64_t)H * W > M3S_MAX_PIXELS) return fail(M3S_ERR_SHAPE, "H * W = %lld exceeds %d", (long long)H * W, M3S_MAX_PIXELS);
    return M3S_OK;
}

m3s_status check_pair(const m3s_pair* A, bool need_desc) {
    if (!A) return fail(M3S_ERR_NULL, "pair is NULL");
    m3s_status s = check_shape(A->H, A->W);
    if (s != M3S_OK) return s;
    if (!A->Xii || !A->Xji) return fail(M3S_ERR_NULL, "Xii and Xji are required");
    if (!aligned(A->Xii, 4) || !aligned(A->Xji, 4)) return fail(M3S_ERR_PARAM, "pointmaps must be 4-byte aligned");
    if (need_desc) {
        if (A->D < 1 || A->D > M3S_MAX_DESC) return fail(M3S_ERR_SHAPE, "D %d outside [1, %d]", A->D, M3S_MAX_DESC);
        if (!A->Dii || !A->Dji) return fail(M3S_ERR_NULL, "Dii and Dji are required");
        if (!aligned(A->Dii, 4) || !aligned(A->Dji, 4)) return fail(M3S_ERR_PARAM, "descriptors must be 4-byte aligned");
        if ((A->Qii == nullptr) != (A->Qji == nullptr)) return fail(M3S_ERR_NULL, "Qii and Qji must both be given or both be NULL");
        if (A->p_init && !aligned(A->p_init, 4)) return fail(M3S_ERR_PARAM, "p_init must be 4-byte aligned");
    }
    return M3S_OK;
}

m3s_status check_outputs(const m3s_outputs* O) {
    if (!O) return fail(M3S_ERR_NULL, "outputs is NULL");
    if (!O->p || !O->idx || !O->valid) return fail(M3S_ERR_NULL, "outputs p, idx and valid are required");
    if (!aligned(O->p, 8)) return fail(M3S_ERR_PARAM, "p must be 8-byte aligned");
    if (!aligned(O->idx, 4) || (O->theta && !aligned(O->theta, 4)) || (O->xhat && !aligned(O->xhat, 4)))
        return fail(M3S_ERR_PARAM, "outputs must be 4-byte aligned");
    return M3S_OK;
}

m3s_status check_bwd(int32_t H, int32_t W, const float* Xii, const float* Xji, const float* p, const uint8_t* valid,
                     const float* grad_p, const float* grad_xhat, const float* grad_Xii, const float* grad_Xji) {
    m3s_status s = check_shape(H, W);
    if (s != M3S_OK) return s;
    if (!Xii || !Xji) return fail(M3S_ERR_NULL, "Xii and Xji are required");
    if (!aligned(Xii, 4) || !aligned(Xji, 4)) return fail(M3S_ERR_PARAM, "pointmaps must be 4-byte aligned");
    if (!p || !valid) return fail(M3S_ERR_NULL, "forward outputs p and valid are required");
    if (!grad_p || !grad_Xii || !grad_Xji) return fail(M3S_ERR_NULL, "grad_p, grad_Xii and grad_Xji are required");
    if (!aligned(p, 4) || !aligned(grad_p, 4) || !aligned(grad_Xii, 4) || !aligned(grad_Xji, 4) ||
        (grad_xhat && !aligned(grad_xhat, 4)))
        return fail(M3S_ERR_PARAM, "gradients must be 4-byte aligned");
    return M3S_OK;
}

m3s::BwdEdgeArgs make_bwd_edge(int32_t H, int32_t W, const float* Xii, const float* Xji, const float* p,
                               const uint8_t* valid, const float* grad_p, const float* grad_xhat, float* grad_Xii,
                               float* grad_Xji) {
    m3s::BwdEdgeArgs B;
    std::memset(&B, 0, sizeof B);
    B.H = H; B.W = W; B.tiles_x = (W + 15) / 16; B.tiles_y = (H + 15) / 16; B.tile_begin = 0;
    B.Xii = Xii; B.Xji = Xji; B.p = p; B.valid = valid; B.grad_p = grad_p; B.grad_xhat = grad_xhat;
    B.dXii = grad_Xii; B.dXji = grad_Xji;
    return B;
}

size_t ray_bytes(int32_t H, int32_t W) { return align_up((size_t)H * W * m3s::kRecBytes); }

// Descriptors go to registers with 16-byte loads when D == 24 and both arrays are 16-byte aligned.
bool desc_in_regs(const m3s_pair* A) {
    return A->D == 24 && aligned(A->Dii, 16) && aligned(A->Dji, 16);
}

EdgeArgs make_edge(const m3s_pair* A, const m3s_outputs* O, const m3s_params* P, int K, int r, const float4* rays) {
    EdgeArgs E;
    std::memset(&E, 0, sizeof E);
    E.H = A->H; E.W = A->W; E.D = A->D; E.K = K; E.r = r; E.levels = P->refine_levels;
    E.lambda0 = P->lambda_init; E.conf_min = P->conf_min; E.max_theta = P->max_theta; E.max_dist = P->max_dist;
    E.Xii = A->Xii; E.Xji = A->Xji; E.Dii = A->Dii; E.Dji = A->Dji;
    E.Qii = A->Qii; E.Qji = A->Qji; E.p_init = A->p_init; E.rays = rays;
    E.p = O->p; E.idx = O->idx; E.valid = O->valid; E.theta = O->theta; E.xhat = O->xhat;
    return E;
}

// Launch override of the calling thread (m3s_debug_set_launch); every field
// -1 means the library's own choice.
thread_local m3s_launch_config g_override = {-1, -1, -1, -1, -1};

// Tile configuration of the single-pair launch and of an untuned batched launch.
int chosen_tile_config() {
    return g_override.tile_config >= 0 ? g_override.tile_config : m3s::kDefaultTileConfig;
}

// Tile-to-XCD band mapping of the single-pair launch (on unless overridden).
bool chosen_xcd_remap() { return g_override.xcd_remap != 0; }

// ---------------------------------------------------------------- batched state

struct Plan {
    std::vector<EdgeArgs> table;     // in launch (tile) order
    std::vector<int32_t> prep_begin;
    int total_tiles = 0, total_prep = 0;
    size_t off_table = 0, off_prep = 0, off_rays = 0, total_bytes = 0;
    bool desc_regs = true;
    int levels = 1;
    std::string signature;
};

// Launch shape of the persistent forward: tile configuration, workgroups,
// and (tile configuration 5) ray-window margin and LM unroll.
struct Launch {
    int tile = m3s::kDefaultTileConfig;
    int grid = 0;
    int margin = m3s::kDefaultMargin;
    int unroll = 1;
};
std::mutex g_cache_mu;
std::map<std::string, Launch> g_tune;               // arch + CU count + shape signature -> best launch
std::map<std::string, hipGraphExec_t> g_graphs;     // signature + ws + launch shape -> graph
std::string g_tune_path;                            // on-disk autotuning cache ("" = none)

// On-disk autotuning cache: one JSON object written by this library,
//   {"format": "m3s-autotune", "version": 1,
//    "entries": {"<key>": [tile, grid, margin, unroll], ...}}
// with keys "<arch>|<CUs>cu|<shape signature>".  Keys hold no quote or
// backslash, so the reader below only has to find strings and integers.
constexpr int kTuneFileVersion = 1;

bool parse_tune_file(const std::string& text, std::map<std::string, Launch>* out) {
    if (text.find("\"format\": \"m3s-autotune\"") == std::string::npos) return false;
    const size_t v = text.find("\"version\":");
    if (v == std::string::npos || std::atoi(text.c_str() + v + 10) != kTuneFileVersion) return false;
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos) return false;
    pos = text.find('{', pos);
    if (pos == std::string::npos) return false;
    ++pos;
    for (;;) {
        const size_t q0 = text.find_first_of("\"}", pos);
        if (q0 == std::string::npos) return false;
        if (text[q0] == '}') return true;
        const size_t q1 = text.find('"', q0 + 1);
        const size_t lb = q1 == std::string::npos ? q1 : text.find('[', q1);
        const size_t rb = lb == std::string::npos ? lb : text.find(']', lb);
        if (rb == std::string::npos) return false;
        Launch L;
        int vals[4];
        const char* c = text.c_str() + lb + 1;
        for (int k = 0; k < 4; ++k) {
            char* end = nullptr;
            long x = std::strtol(c, &end, 10);
            if (end == c || x < 0 || x > (1 << 20)) return false;
            vals[k] = (int)x;
            c = end;
            while (*c == ' ' || *c == ',') ++c;
        }
        L.tile = vals[0]; L.grid = vals[1]; L.margin = vals[2]; L.unroll = vals[3];
        if (L.tile >= m3s::kNumTileConfigs || L.grid < 1 || L.margin < m3s::kMarginMin || L.margin > m3s::kMarginMax ||
            L.unroll < 1 || L.unroll > m3s::kUnrollMax)
            return false;
        (*out)[text.substr(q0 + 1, q1 - q0 - 1)] = L;
        pos = rb + 1;
    }
}

// Writes g_tune to g_tune_path (caller holds g_cache_mu): a temporary file
// renamed over the old one, so a reader never sees half a file.
bool save_tune_file() {
    if (g_tune_path.empty()) return true;
    const std::string tmp = g_tune_path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\"format\": \"m3s-autotune\", \"version\": %d,\n \"entries\": {", kTuneFileVersion);
    bool first = true;
    for (const auto& kv : g_tune) {
        std::fprintf(f, "%s\n  \"%s\": [%d, %d, %d, %d]", first ? "" : ",", kv.first.c_str(), kv.second.tile,
                     kv.second.grid, kv.second.margin, kv.second.unroll);
        first = false;
    }
    std::fprintf(f, "\n }}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), g_tune_path.c_str()) == 0;
}

m3s_status plan_batched(const m3s_edge* edges, int32_t n, const m3s_params* P, int tile_config, Plan* plan) {
    if (!edges) return fail(M3S_ERR_NULL, "edges is NULL");
    if (n < 1 || n > (1 << 20)) return fail(M3S_ERR_SHAPE, "n_edges %d outside [1, 2^20]", n);
    m3s_status s = check_params(P);
    if (s != M3S_OK) return s;
    // Heaviest edges first (queries x (iterations + window)), so the work queue
    // ends on small tiles.
    std::vector<int> order(n);
    std::vector<double> cost(n);
    for (int e = 0; e < n; ++e) {
        const m3s_edge& E = edges[e];
        s = check_pair(&E.in, true);
        if (s != M3S_OK) return fail(s, "edge %d: %s", e, g_last_error.c_str());
        s = check_outputs(&E.out);
        if (s != M3S_OK) return fail(s, "edge %d: %s", e, g_last_error.c_str());
        int K = E.max_iter >= 0 ? E.max_iter : P->max_iter;
        int r = E.refine_radius >= 0 ? E.refine_radius : P->refine_radius;
        if (K > M3S_MAX_ITER) return fail(M3S_ERR_PARAM, "edge %d: max_iter %d > %d", e, K, M3S_MAX_ITER);
        if (r > M3S_MAX_RADIUS) return fail(M3S_ERR_PARAM, "edge %d: refine_radius %d > %d", e, r, M3S_MAX_RADIUS);
        order[e] = e;
        cost[e] = (double)E.in.H * E.in.W * (20.0 * (K + 1) + (double)E.in.D * (2 * r + 1) * (2 * r + 1));
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    int tx, ty;
    m3s::tile_shape(tile_config, &tx, &ty);
    plan->table.clear();
    plan->prep_begin.clear();
    plan->desc_regs = true;
    size_t off = align_up(sizeof(int32_t));
    plan->off_table = off;
    off += align_up(sizeof(EdgeArgs) * (size_t)n);
    plan->off_prep = off;
    off += align_up(sizeof(int32_t) * (size_t)n);
    plan->off_rays = off;
    int64_t tiles = 0, prep = 0;
    std::string sig;
    char buf[96];
    for (int k = 0; k < n; ++k) {
        const m3s_edge& E = edges[order[k]];
        int K = E.max_iter >= 0 ? E.max_iter : P->max_iter;
        int r = E.refine_radius >= 0 ? E.refine_radius : P->refine_radius;
        EdgeArgs A = make_edge(&E.in, &E.out, P, K, r, nullptr);
        A.rays = reinterpret_cast<const float4*>(off);  // offset; rebased onto ws by the caller
        off += ray_bytes(E.in.H, E.in.W);
        A.tiles_x = (E.in.W + tx - 1) / tx;
        A.tiles_y = (E.in.H + ty - 1) / ty;
        A.tile_begin = (int32_t)tiles;
        tiles += (int64_t)A.tiles_x * A.tiles_y;
        plan->prep_begin.push_back((int32_t)prep);
        prep += m3s::prep_tiles(E.in.H, E.in.W);
        if (tiles > INT32_MAX / 2 || prep > INT32_MAX / 2) return fail(M3S_ERR_SHAPE, "batch too large");
        if (!desc_in_regs(&E.in)) plan->desc_regs = false;
        plan->table.push_back(A);
        snprintf(buf, sizeof buf, "%d,%d,%d,%d,%d,%d,%d;", order[k], E.in.H, E.in.W, E.in.D, K, r,
                 (E.in.Qii ? 1 : 0) | (E.in.p_init ? 2 : 0) | (E.out.theta ? 4 : 0) | (E.out.xhat ? 8 : 0));
        sig += buf;
    }
    plan->total_tiles = (int)tiles;
    plan->total_prep = (int)prep;
    plan->total_bytes = off;
    plan->levels = P->refine_levels;
    plan->signature = sig + (plan->desc_regs ? "R" : "G") + "L" + std::to_string(P->refine_levels);
    return M3S_OK;
}

// Host -> device copies of the edge tables: the table is written into a
// pinned staging buffer and a small kernel on the stream reads it from there
// (a DMA copy starts later in the stream than a kernel does, and from
// pageable memory hipMemcpyAsync may also wait for the stream).  Each device
// has a ring of kStageSlots slots; a slot is reused only after the kernel
// that last read it has completed (its event).
constexpr int kStageSlots = 8;
struct StageSlot {
    char* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};
struct StageRing {
    StageSlot slot[kStageSlots];
    int next = 0;
};
std::mutex g_stage_mu;
std::map<int, StageRing> g_stage;

m3s_status staged_copy(void* dst, const void* src, size_t bytes, hipStream_t s, const char* what) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_stage_mu);
    StageRing& ring = g_stage[dev];
    StageSlot& sl = ring.slot[ring.next];
    ring.next = (ring.next + 1) % kStageSlots;
    if (sl.done && (e = hipEventSynchronize(sl.done)) != hipSuccess) return hip_fail(e, "hipEventSynchronize(staging)");
    if (sl.cap < bytes) {
        if (sl.host && (e = hipHostFree(sl.host)) != hipSuccess) return hip_fail(e, "hipHostFree(staging)");
        sl.host = nullptr;
        sl.cap = 0;
        const size_t cap = std::max(bytes, (size_t)4096);
        if ((e = hipHostMalloc((void**)&sl.host, cap, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "hipHostMalloc(staging)");
        sl.cap = cap;
    }
    if (!sl.done && (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate(staging)");
    std::memcpy(sl.host, src, bytes);
    if (bytes % 4 || reinterpret_cast<uintptr_t>(dst) % 4) return fail(M3S_ERR_HIP, "%s: unaligned table copy", what);
    if ((e = m3s::launch_host_copy(dst, sl.host, bytes, s)) != hipSuccess) return hip_fail(e, what);
    if ((e = hipEventRecord(sl.done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord(staging)");
    return M3S_OK;
}

// Rebase the table onto the workspace and copy it and prep_begin to the
// device in one copy (the workspace bytes [off_table, off_prep + prep size)).
m3s_status upload_plan(Plan& plan, char* ws, hipStream_t s) {
    for (EdgeArgs& A : plan.table) A.rays = reinterpret_cast<const float4*>(ws + reinterpret_cast<uintptr_t>(A.rays));
    const size_t tb = sizeof(EdgeArgs) * plan.table.size(), pb = sizeof(int32_t) * plan.prep_begin.size();
    std::vector<char> image(plan.off_prep - plan.off_table + pb, 0);
    std::memcpy(image.data(), plan.table.data(), tb);
    std::memcpy(image.data() + (plan.off_prep - plan.off_table), plan.prep_begin.data(), pb);
    return staged_copy(ws + plan.off_table, image.data(), image.size(), s, "edge table copy");
}

hipError_t run_batched(const Plan& plan, char* ws, const Launch& L, hipStream_t s) {
    return m3s::launch_batched(reinterpret_cast<const EdgeArgs*>(ws + plan.off_table),
                               reinterpret_cast<const int32_t*>(ws + plan.off_prep), (int)plan.table.size(),
                               plan.total_prep, plan.total_tiles, reinterpret_cast<int32_t*>(ws), L.tile,
                               std::max(1, std::min(L.grid, plan.total_tiles)), L.margin, L.unroll, plan.levels,
                               plan.desc_regs, s);
}

// Times every candidate launch of one batch (warm-up plus three timed
// launches each) and returns the fastest: first the tile configuration x
// grid (1, 2, 4 or 8 workgroups per CU) with the default margin and unroll,
// then, for the fp16 configuration, ray-window margin x LM unroll at its best
// grid.  Synchronises the stream; every candidate writes the same outputs.
m3s_status autotune(const m3s_edge* edges, int32_t n, const m3s_params* P, char* W, int cus, hipStream_t st,
                    Launch* best_out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return fail(M3S_ERR_HIP, "hipEventCreate failed");
    }
    float best_ms = INFINITY;
    Launch best;
    m3s_status s = M3S_OK;
    auto time_it = [&](const Plan& plan, const Launch& L) -> bool {
        hipError_t e = run_batched(plan, W, L, st);  // warm-up
        float sum = 0.f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            hipEventRecord(e0, st);
            e = run_batched(plan, W, L, st);
            hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            sum += ms;
        }
        if (e != hipSuccess) { s = hip_fail(e, "autotune launch"); return false; }
        if (sum < best_ms) { best_ms = sum; best = L; }
        return true;
    };
    const int mults[] = {1, 2, 4, 8};
    for (int tc = 0; tc < m3s::kNumTileConfigs && s == M3S_OK; ++tc) {
        Plan plan;
        if ((s = plan_batched(edges, n, P, tc, &plan)) != M3S_OK) break;
        if ((s = upload_plan(plan, W, st)) != M3S_OK) break;
        for (int mult : mults) {
            Launch L;
            L.tile = tc;
            L.grid = std::max(1, std::min(cus * mult, plan.total_tiles));  // the grid the launch really has
            if (!time_it(plan, L)) break;
        }
    }
    if (s == M3S_OK && best.tile == 5) {
        Plan plan;
        if ((s = plan_batched(edges, n, P, best.tile, &plan)) == M3S_OK && (s = upload_plan(plan, W, st)) == M3S_OK) {
            const Launch base = best;
            for (int m = m3s::kMarginMin; m <= m3s::kMarginMax && s == M3S_OK; ++m)
                for (int u = 1; u <= m3s::kUnrollMax; ++u) {
                    if (m == base.margin && u == base.unroll) continue;
                    Launch L = base;
                    L.margin = m; L.unroll = u;
                    if (!time_it(plan, L)) break;
                }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s == M3S_OK) *best_out = best;
    return s;
}

// ---------------------------------------------------------------- kernel timing

struct TimedLaunch { std::string name; hipEvent_t e0, e1; };
std::mutex g_timer_mu;
bool g_timer_on = false;
std::vector<TimedLaunch> g_timed;          // recorded, not yet read
std::vector<hipEvent_t> g_event_pool;
std::map<std::string, std::pair<double, int64_t>> g_timer_totals;
thread_local std::string g_timer_name;
thread_local hipEvent_t g_timer_e0 = nullptr;
thread_local bool g_timer_suppressed = false;  // set around m3s_match_fwd_noalloc (no event creation)

hipEvent_t pooled_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool capturing(hipStream_t s) {
    if (s == nullptr) return false;  // the null stream is never captured
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return true;
    return st != hipStreamCaptureStatusNone;
}

}  // namespace

namespace m3s {

void timer_begin(const char* name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    g_timer_e0 = nullptr;
    if (!g_timer_on || g_timer_suppressed || capturing(s)) return;
    hipEvent_t e0 = pooled_event();
    if (!e0) return;
    if (hipEventRecord(e0, s) != hipSuccess) { g_event_pool.push_back(e0); return; }
    g_timer_e0 = e0;
    g_timer_name = name;
}

void timer_end(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    if (!g_timer_e0) return;
    hipEvent_t e1 = pooled_event();
    if (e1 && hipEventRecord(e1, s) == hipSuccess) {
        g_timed.push_back({g_timer_name, g_timer_e0, e1});
    } else {
        g_event_pool.push_back(g_timer_e0);
        if (e1) g_event_pool.push_back(e1);
    }
    g_timer_e0 = nullptr;
}

}  // namespace m3s

namespace {

m3s_status drain_timings() {
    for (TimedLaunch& t : g_timed) {
        hipError_t e = hipEventSynchronize(t.e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.e0, t.e1);
        if (e != hipSuccess) return hip_fail(e, "timing events");
        auto& tot = g_timer_totals[t.name];
        tot.first += ms;
        tot.second += 1;
        g_event_pool.push_back(t.e0);
        g_event_pool.push_back(t.e1);
    }
    g_timed.clear();
    return M3S_OK;
}

}  // namespace

// ---------------------------------------------------------------- no-allocation scratch
//
// Ray records for m3s_match_fwd_noalloc live in this file-scope device array
// (one copy per GPU, held until the process ends).  Host code never passes
// the array's name to a kernel: on the host it is only a stand-in for the
// symbol.  The device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept here.
namespace m3s {
__device__ __align__(256) float4 scratch[(size_t)M3S_NOALLOC_MAX_PIXELS * kRecBytes / sizeof(float4)];
}  // namespace m3s

namespace {

std::mutex g_scratch_mu;
std::map<int, float4*> g_scratch_ptr;

m3s_status scratch_of_device(int dev, float4** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return M3S_OK;
    }
    float4* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(m3s::scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (ptr == nullptr || !aligned(ptr, kAlign)) return fail(M3S_ERR_HIP, "scratch address is not 256-byte aligned");
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return M3S_OK;
}

}  // namespace

extern "C" {

void m3s_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    g_timer_on = on != 0;
}

m3s_status m3s_timing_read(const char* name, double* total_ms, int64_t* launches) {
    if (!name || !total_ms || !launches) return fail(M3S_ERR_NULL, "name, total_ms and launches are required");
    std::lock_guard<std::mutex> lk(g_timer_mu);
    m3s_status s = drain_timings();
    if (s != M3S_OK) return s;
    auto it = g_timer_totals.find(name);
    *total_ms = it == g_timer_totals.end() ? 0.0 : it->second.first;
    *launches = it == g_timer_totals.end() ? 0 : it->second.second;
    return M3S_OK;
}

void m3s_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    drain_timings();
    g_timer_totals.clear();
}


void m3s_default_params(m3s_params* P) {
    if (!P) return;
    P->max_iter = 10;
    P->lambda_init = 1e-8f;
    P->refine_radius = 3;
    P->refine_levels = 1;
    P->conf_min = 1.5f;
    P->max_theta = 1e-4f;
    P->max_dist = INFINITY;
}

size_t m3s_workspace_bytes(const m3s_pair* pair, const m3s_params*) {
    if (!pair || pair->H < 2 || pair->W < 2 || (int64_t)pair->H * pair->W > M3S_MAX_PIXELS) return 0;
    return ray_bytes(pair->H, pair->W);
}

m3s_status m3s_match_fwd(const m3s_pair* pair, const m3s_params* params, const m3s_outputs* out, void* ws,
                         size_t ws_bytes, void* stream) {
    m3s_params defaults;
    m3s_default_params(&defaults);
    const m3s_params* P = params ? params : &defaults;
    m3s_status s = check_params(P);
    if (s != M3S_OK) return s;
    if ((s = check_pair(pair, true)) != M3S_OK) return s;
    if ((s = check_outputs(out)) != M3S_OK) return s;
    size_t need = ray_bytes(pair->H, pair->W);
    if (!ws || !aligned(ws, kAlign) || ws_bytes < need)
        return fail(M3S_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need, ws_bytes);
    int dev;
    DeviceInfo info;
    if ((s = current_device(&dev, &info)) != M3S_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float4* rays = reinterpret_cast<float4*>(ws);
    EdgeArgs A = make_edge(pair, out, P, P->max_iter, P->refine_radius, rays);
    hipError_t e = m3s::launch_prep(pair->Xii, rays, pair->H, pair->W, st);
    if (e != hipSuccess) return hip_fail(e, "prep launch");
    e = m3s::launch_fwd(A, chosen_tile_config(), desc_in_regs(pair), chosen_xcd_remap(), st);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    g_last_error.clear();
    return M3S_OK;
}

m3s_status m3s_match_fwd_noalloc(const m3s_pair* pair, const m3s_params* params, const m3s_outputs* out,
                                 void* stream) {
    m3s_params defaults;
    m3s_default_params(&defaults);
    const m3s_params* P = params ? params : &defaults;
    m3s_status s = check_params(P);
    if (s != M3S_OK) return s;
    if ((s = check_pair(pair, true)) != M3S_OK) return s;
    if ((s = check_outputs(out)) != M3S_OK) return s;
    if ((int64_t)pair->H * pair->W > M3S_NOALLOC_MAX_PIXELS)
        return fail(M3S_ERR_SHAPE, "H * W = %lld exceeds the no-allocation limit M3S_NOALLOC_MAX_PIXELS = %d",
                    (long long)pair->H * pair->W, M3S_NOALLOC_MAX_PIXELS);
    int dev;
    DeviceInfo info;
    if ((s = current_device(&dev, &info)) != M3S_OK) return s;
    float4* rays = nullptr;
    if ((s = scratch_of_device(dev, &rays)) != M3S_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    EdgeArgs A = make_edge(pair, out, P, P->max_iter, P->refine_radius, rays);
    g_timer_suppressed = true;
    hipError_t e = m3s::launch_prep(pair->Xii, rays, pair->H, pair->W, st);
    if (e == hipSuccess) e = m3s::launch_fwd(A, chosen_tile_config(), desc_in_regs(pair), chosen_xcd_remap(), st);
    g_timer_suppressed = false;
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    g_last_error.clear();
    return M3S_OK;
}

m3s_status m3s_match_bwd(const m3s_pair* pair, const m3s_outputs* fwd, const float* grad_p, const float* grad_xhat,
                         float* grad_Xii, float* grad_Xji, void* stream) {
    if (!pair) return fail(M3S_ERR_NULL, "pair is NULL");
    if (!fwd) return fail(M3S_ERR_NULL, "forward outputs p and valid are required");
    m3s_status s = check_bwd(pair->H, pair->W, pair->Xii, pair->Xji, fwd->p, fwd->valid, grad_p, grad_xhat, grad_Xii,
                             grad_Xji);
    if (s != M3S_OK) return s;
    int dev;
    DeviceInfo info;
    if ((s = current_device(&dev, &info)) != M3S_OK) return s;
    hipError_t e = m3s::launch_bwd(make_bwd_edge(pair->H, pair->W, pair->Xii, pair->Xji, fwd->p, fwd->valid, grad_p,
                                                 grad_xhat, grad_Xii, grad_Xji),
                                   reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    g_last_error.clear();
    return M3S_OK;
}

size_t m3s_bwd_batched_workspace_bytes(int32_t n_edges) {
    if (n_edges < 1 || n_edges > (1 << 20)) return 0;
    return align_up(sizeof(m3s::BwdEdgeArgs) * (size_t)n_edges);
}

m3s_status m3s_match_bwd_batched(const m3s_bwd_edge* edges, int32_t n_edges, uint32_t flags, void* ws,
                                 size_t ws_bytes, void* stream) {
    if (!edges) return fail(M3S_ERR_NULL, "edges is NULL");
    if (n_edges < 1 || n_edges > (1 << 20)) return fail(M3S_ERR_SHAPE, "n_edges %d outside [1, 2^20]", n_edges);
    if (flags & ~(uint32_t)(M3S_BATCH_GRAPH | M3S_BWD_ACCUMULATE))
        return fail(M3S_ERR_UNSUPPORTED, "unknown flags 0x%x", flags);
    const bool zero = !(flags & M3S_BWD_ACCUMULATE);
    std::vector<m3s::BwdEdgeArgs> table((size_t)n_edges);
    int64_t tiles = 0;
    long max_px = 0;
    std::string sig = "B";
    char buf[64];
    for (int k = 0; k < n_edges; ++k) {
        const m3s_bwd_edge& E = edges[k];
        m3s_status s = check_bwd(E.H, E.W, E.Xii, E.Xji, E.p, E.valid, E.grad_p, E.grad_xhat, E.grad_Xii, E.grad_Xji);
        if (s != M3S_OK) return fail(s, "edge %d: %s", k, g_last_error.c_str());
        table[k] = make_bwd_edge(E.H, E.W, E.Xii, E.Xji, E.p, E.valid, E.grad_p, E.grad_xhat, E.grad_Xii, E.grad_Xji);
        table[k].tile_begin = (int32_t)tiles;
        tiles += (int64_t)table[k].tiles_x * table[k].tiles_y;
        if (tiles > INT32_MAX / 2) return fail(M3S_ERR_SHAPE, "batch too large");
        max_px = std::max(max_px, (long)E.H * E.W);
        snprintf(buf, sizeof buf, "%d,%d;", E.H, E.W);
        sig += buf;
    }
    const size_t need = m3s_bwd_batched_workspace_bytes(n_edges);
    if (!ws || !aligned(ws, kAlign) || ws_bytes < need)
        return fail(M3S_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need, ws_bytes);
    int dev;
    DeviceInfo info;
    m3s_status s = current_device(&dev, &info);
    if (s != M3S_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (capturing(st))
        return fail(M3S_ERR_UNSUPPORTED,
                    "m3s_match_bwd_batched cannot be captured: it copies its edge table from host memory before every "
                    "launch; M3S_BATCH_GRAPH gives a library-managed graph instead");
    char* W = reinterpret_cast<char*>(ws);
    auto* dtable = reinterpret_cast<m3s::BwdEdgeArgs*>(W);
    if ((s = staged_copy(dtable, table.data(), sizeof(m3s::BwdEdgeArgs) * table.size(), st,
                         "hipMemcpyAsync(backward edge table)")) != M3S_OK)
        return s;
    hipError_t e = hipSuccess;
    // 32 workgroups per CU, each taking every grid-th tile of its XCD's band
    // (measured on the 16-edge 512x384 workload: 79 us, against 85 us with 12
    // per CU, 91 us with 8 and 81 us with one workgroup per tile).
    const int grid = std::max(1, std::min((int)tiles, g_override.grid > 0 ? g_override.grid : info.cus * 32));
    if ((flags & M3S_BATCH_GRAPH) && st != nullptr) {
        std::string gkey = std::to_string(dev) + "|" + sig + "|" + std::to_string(reinterpret_cast<uintptr_t>(ws)) +
                           "|" + std::to_string(grid) + (zero ? "|z" : "|a");
        hipGraphExec_t exec = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_graphs.find(gkey);
            if (it != g_graphs.end()) exec = it->second;
        }
        if (!exec) {
            e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le = m3s::launch_bwd_batched(dtable, n_edges, max_px, (int)tiles, grid, zero, st);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(st, &graph);
            if (le != hipSuccess) { if (graph) hipGraphDestroy(graph); return hip_fail(le, "captured launch"); }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_graphs[gkey] = exec;
        }
        m3s::timer_begin("batched_bwd_graph", st);
        e = hipGraphLaunch(exec, st);
        m3s::timer_end(st);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        e = m3s::launch_bwd_batched(dtable, n_edges, max_px, (int)tiles, grid, zero, st);
        if (e != hipSuccess) return hip_fail(e, "batched backward launch");
    }
    g_last_error.clear();
    return M3S_OK;
}

size_t m3s_stats_workspace_bytes(int32_t H, int32_t W) {
    if (H < 2 || W < 2 || (int64_t)H * W > M3S_MAX_PIXELS) return 0;
    return align_up(((size_t)H * W + 31) / 32 * sizeof(uint32_t));
}

m3s_status m3s_match_stats(const m3s_outputs* fwd, int32_t H, int32_t W, int32_t* counts, void* ws, size_t ws_bytes,
                           void* stream) {
    m3s_status s = check_shape(H, W);
    if (s != M3S_OK) return s;
    if (!fwd || !fwd->idx || !fwd->valid || !counts) return fail(M3S_ERR_NULL, "idx, valid and counts are required");
    if (!aligned(fwd->idx, 4) || !aligned(counts, 4)) return fail(M3S_ERR_PARAM, "idx and counts must be 4-byte aligned");
    size_t need = m3s_stats_workspace_bytes(H, W);
    if (!ws || !aligned(ws, kAlign) || ws_bytes < need)
        return fail(M3S_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need, ws_bytes);
    int dev;
    DeviceInfo info;
    if ((s = current_device(&dev, &info)) != M3S_OK) return s;
    hipError_t e = m3s::launch_stats(fwd->idx, fwd->valid, H, W, reinterpret_cast<uint32_t*>(ws), counts,
                                     reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "statistics launch");
    g_last_error.clear();
    return M3S_OK;
}

void m3s_default_track_params(m3s_track_params* P) {
    if (!P) return;
    P->iters = 10;
    P->q_min = 1.5f;
    P->sigma_ray = 0.003f;
    P->sigma_dist = 0.1f;
    P->huber = 1.345f;
}

size_t m3s_track_workspace_bytes(int32_t H, int32_t W) {
    if (H < 2 || W < 2 || (int64_t)H * W > M3S_MAX_PIXELS) return 0;
    return align_up(m3s::track_workspace_bytes(H * W));
}

m3s_status m3s_track_pose(const m3s_track_problem* prob, const m3s_track_params* params, float* T, float* info,
                          void* ws, size_t ws_bytes, void* stream) {
    m3s_track_params defaults;
    m3s_default_track_params(&defaults);
    const m3s_track_params* P = params ? params : &defaults;
    if (!prob) return fail(M3S_ERR_NULL, "problem is NULL");
    m3s_status s = check_shape(prob->H, prob->W);
    if (s != M3S_OK) return s;
    if (!prob->Xk || !prob->Xf || !prob->idx || !prob->valid || !prob->Qf || !prob->Qk)
        return fail(M3S_ERR_NULL, "Xk, Xf, idx, valid, Qf and Qk are required");
    if (!T) return fail(M3S_ERR_NULL, "T is required");
    if (!aligned(prob->Xk, 4) || !aligned(prob->Xf, 4) || !aligned(prob->idx, 4) || !aligned(prob->Qf, 4) ||
        !aligned(prob->Qk, 4) || !aligned(T, 4) || (info && !aligned(info, 4)))
        return fail(M3S_ERR_PARAM, "arrays must be 4-byte aligned");
    if (P->iters < 0 || P->iters > M3S_MAX_ITER) return fail(M3S_ERR_PARAM, "iters %d outside [0, %d]", P->iters, M3S_MAX_ITER);
    if (!std::isfinite(P->q_min)) return fail(M3S_ERR_PARAM, "q_min must be finite");
    if (std::isnan(P->sigma_ray) || !(P->sigma_ray > 0.f)) return fail(M3S_ERR_PARAM, "sigma_ray must be > 0");
    if (std::isnan(P->sigma_dist) || !(P->sigma_dist > 0.f)) return fail(M3S_ERR_PARAM, "sigma_dist must be > 0");
    if (std::isnan(P->huber) || !(P->huber > 0.f)) return fail(M3S_ERR_PARAM, "huber must be > 0");
    const size_t need = m3s_track_workspace_bytes(prob->H, prob->W);
    if (!ws || !aligned(ws, kAlign) || ws_bytes < need)
        return fail(M3S_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need, ws_bytes);
    int dev;
    DeviceInfo info_dev;
    if ((s = current_device(&dev, &info_dev)) != M3S_OK) return s;
    hipError_t e = m3s::launch_track(prob->H * prob->W, prob->Xk, prob->Xf, prob->idx, prob->valid, prob->Qf, prob->Qk,
                                     P->q_min, P->sigma_ray, P->sigma_dist, P->huber, P->iters, T, info, ws,
                                     reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "tracking launch");
    g_last_error.clear();
    return M3S_OK;
}

m3s_status m3s_fuse_pointmap(const m3s_fuse_problem* prob, const float* T, void* stream) {
    if (!prob) return fail(M3S_ERR_NULL, "problem is NULL");
    m3s_status s = check_shape(prob->H, prob->W);
    if (s != M3S_OK) return s;
    if (!prob->Xc || !prob->Cc || !prob->X || !prob->C || !T) return fail(M3S_ERR_NULL, "Xc, Cc, X, C and T are required");
    if (!aligned(prob->Xc, 4) || !aligned(prob->Cc, 4) || !aligned(prob->X, 4) || !aligned(prob->C, 4) || !aligned(T, 4))
        return fail(M3S_ERR_PARAM, "arrays must be 4-byte aligned");
    int dev;
    DeviceInfo info_dev;
    if ((s = current_device(&dev, &info_dev)) != M3S_OK) return s;
    hipError_t e = m3s::launch_fuse(prob->H * prob->W, T, prob->Xc, prob->Cc, prob->X, prob->C,
                                    reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "fusion launch");
    g_last_error.clear();
    return M3S_OK;
}

void m3s_default_backend_params(m3s_backend_params* P) {
    if (!P) return;
    P->iters = 10;
    P->q_min = 1.5f;
    P->sigma_ray = 0.003f;
    P->sigma_dist = 0.1f;
    P->huber = 1.345f;
    P->step_tol = 0.0;
}

size_t m3s_backend_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t E) {
    if (N < 2 || N > M3S_MAX_KEYFRAMES || E < 1 || E > M3S_MAX_EDGES || H < 2 || W < 2 ||
        (int64_t)H * W > M3S_MAX_PIXELS)
        return 0;
    return align_up(m3s::backend_workspace_bytes(N, H * W, E));
}

m3s_status m3s_backend_gn(const m3s_backend_problem* prob, const m3s_backend_params* params, float* T_WC,
                          float* info, void* ws, size_t ws_bytes, void* stream) {
    m3s_backend_params defaults;
    m3s_default_backend_params(&defaults);
    const m3s_backend_params* P = params ? params : &defaults;
    if (!prob) return fail(M3S_ERR_NULL, "problem is NULL");
    m3s_status s = check_shape(prob->H, prob->W);
    if (s != M3S_OK) return s;
    if (prob->N < 2 || prob->N > M3S_MAX_KEYFRAMES)
        return fail(M3S_ERR_SHAPE, "N %d outside [2, %d]", prob->N, M3S_MAX_KEYFRAMES);
    if (prob->E < 1 || prob->E > M3S_MAX_EDGES) return fail(M3S_ERR_SHAPE, "E %d outside [1, %d]", prob->E, M3S_MAX_EDGES);
    if ((int64_t)prob->N * prob->H * prob->W * 3 > INT32_MAX || (int64_t)prob->E * prob->H * prob->W > INT32_MAX)
        return fail(M3S_ERR_SHAPE, "N * H * W * 3 and E * H * W must stay below 2^31");
    if (!prob->Xc || !prob->Q || !prob->edges || !prob->idx || !prob->valid || !T_WC)
        return fail(M3S_ERR_NULL, "Xc, Q, edges, idx, valid and T_WC are required");
    if (!aligned(prob->Xc, 4) || !aligned(prob->Q, 4) || !aligned(prob->edges, 4) || !aligned(prob->idx, 4) ||
        !aligned(T_WC, 4) || (info && !aligned(info, 4)))
        return fail(M3S_ERR_PARAM, "arrays must be 4-byte aligned");
    if (P->iters < 0 || P->iters > M3S_MAX_ITER) return fail(M3S_ERR_PARAM, "iters %d outside [0, %d]", P->iters, M3S_MAX_ITER);
    if (!std::isfinite(P->q_min)) return fail(M3S_ERR_PARAM, "q_min must be finite");
    if (std::isnan(P->sigma_ray) || !(P->sigma_ray > 0.f)) return fail(M3S_ERR_PARAM, "sigma_ray must be > 0");
    if (std::isnan(P->sigma_dist) || !(P->sigma_dist > 0.f)) return fail(M3S_ERR_PARAM, "sigma_dist must be > 0");
    if (std::isnan(P->huber) || !(P->huber > 0.f)) return fail(M3S_ERR_PARAM, "huber must be > 0");
    if (std::isnan(P->step_tol) || P->step_tol < 0.0) return fail(M3S_ERR_PARAM, "step_tol must be >= 0");
    const size_t need = m3s_backend_workspace_bytes(prob->N, prob->H, prob->W, prob->E);
    if (!ws || !aligned(ws, kAlign) || ws_bytes < need)
        return fail(M3S_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", need, ws_bytes);
    int dev;
    DeviceInfo info_dev;
    if ((s = current_device(&dev, &info_dev)) != M3S_OK) return s;
    hipError_t e = m3s::launch_backend(prob->N, prob->H * prob->W, prob->E, prob->Xc, prob->Q, prob->edges, prob->idx,
                                       prob->valid, P->q_min, P->sigma_ray, P->sigma_dist, P->huber, P->iters,
                                       P->step_tol, T_WC, info, ws, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "backend launch");
    g_last_error.clear();
    return M3S_OK;
}

size_t m3s_batched_workspace_bytes(const m3s_edge* edges, int32_t n_edges, const m3s_params* common) {
    m3s_params defaults;
    m3s_default_params(&defaults);
    Plan plan;
    std::string saved = g_last_error;
    m3s_status s = plan_batched(edges, n_edges, common ? common : &defaults, 0, &plan);
    g_last_error = saved;
    return s == M3S_OK ? plan.total_bytes : 0;
}

m3s_status m3s_match_batched(const m3s_edge* edges, int32_t n_edges, const m3s_params* common, uint32_t flags,
                             void* ws, size_t ws_bytes, void* stream) {
    m3s_params defaults;
    m3s_default_params(&defaults);
    const m3s_params* P = common ? common : &defaults;
    if (flags & ~(uint32_t)(M3S_BATCH_GRAPH | M3S_BATCH_AUTOTUNE))
        return fail(M3S_ERR_UNSUPPORTED, "unknown flags 0x%x", flags);
    Launch L;
    L.tile = chosen_tile_config();
    if (g_override.ray_margin > 0) L.margin = std::min(std::max(g_override.ray_margin, m3s::kMarginMin), m3s::kMarginMax);
    if (g_override.lm_unroll > 0) L.unroll = std::min(g_override.lm_unroll, m3s::kUnrollMax);
    const bool overridden = g_override.tile_config >= 0 || g_override.grid > 0 || g_override.ray_margin > 0 ||
                            g_override.lm_unroll > 0;
    Plan plan;
    m3s_status s = plan_batched(edges, n_edges, P, L.tile, &plan);
    if (s != M3S_OK) return s;
    if (!ws || !aligned(ws, kAlign) || ws_bytes < plan.total_bytes)
        return fail(M3S_ERR_WORKSPACE, "workspace must be 256-byte aligned and >= %zu bytes (got %zu)", plan.total_bytes,
                    ws_bytes);
    int dev;
    DeviceInfo info;
    if ((s = current_device(&dev, &info)) != M3S_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (capturing(st))
        return fail(M3S_ERR_UNSUPPORTED,
                    "m3s_match_batched cannot be captured: it copies its edge table from host memory before every "
                    "launch; M3S_BATCH_GRAPH gives a library-managed graph instead");
    char* W = reinterpret_cast<char*>(ws);
    const std::string tune_key = info.arch + "|" + std::to_string(info.cus) + "cu|" + plan.signature;

    L.grid = g_override.grid > 0 ? g_override.grid : info.cus * 4;
    if ((flags & M3S_BATCH_AUTOTUNE) && !overridden) {
        Launch tr;
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_tune.find(tune_key);
            if (it != g_tune.end()) { tr = it->second; have = true; }
        }
        if (!have) {
            if ((s = autotune(edges, n_edges, P, W, info.cus, st, &tr)) != M3S_OK) return s;
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_tune[tune_key] = tr;
            if (!save_tune_file()) return fail(M3S_ERR_PARAM, "cannot write the autotuning cache %s", g_tune_path.c_str());
        }
        if (tr.tile != L.tile && (s = plan_batched(edges, n_edges, P, tr.tile, &plan)) != M3S_OK) return s;
        L = tr;
    }
    L.grid = std::max(1, std::min(L.grid, plan.total_tiles));
    if ((s = upload_plan(plan, W, st)) != M3S_OK) return s;
    g_last_grid = L.grid;
    g_last_tile = L.tile;
    g_last_margin = L.margin;
    g_last_unroll = L.unroll;

    if ((flags & M3S_BATCH_GRAPH) && st != nullptr) {
        char lb[64];
        snprintf(lb, sizeof lb, "|%d,%d,%d,%d", L.tile, L.grid, L.margin, L.unroll);
        std::string gkey = std::to_string(dev) + "|" + tune_key + "|" + std::to_string(reinterpret_cast<uintptr_t>(ws)) + lb;
        hipGraphExec_t exec = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_graphs.find(gkey);
            if (it != g_graphs.end()) exec = it->second;
        }
        if (!exec) {
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le = run_batched(plan, W, L, st);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(st, &graph);
            if (le != hipSuccess) { if (graph) hipGraphDestroy(graph); return hip_fail(le, "captured launch"); }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_graphs[gkey] = exec;
        }
        m3s::timer_begin("batched_graph", st);
        hipError_t e = hipGraphLaunch(exec, st);
        m3s::timer_end(st);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        hipError_t e = run_batched(plan, W, L, st);
        if (e != hipSuccess) return hip_fail(e, "batched launch");
    }
    g_last_error.clear();
    return M3S_OK;
}

void m3s_debug_set_launch(const m3s_launch_config* cfg) {
    if (cfg) {
        g_override = *cfg;
        if (g_override.tile_config >= m3s::kNumTileConfigs) g_override.tile_config = -1;
    } else {
        g_override = m3s_launch_config{-1, -1, -1, -1, -1};
    }
}

m3s_status m3s_set_tune_cache(const char* path) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (!path || !path[0]) {
        g_tune_path.clear();
        return M3S_OK;
    }
    std::map<std::string, Launch> loaded;
    if (FILE* f = std::fopen(path, "r")) {
        std::string text;
        char buf[4096];
        size_t got;
        while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
        std::fclose(f);
        if (!parse_tune_file(text, &loaded))
            return fail(M3S_ERR_PARAM, "%s is not an m3s autotuning cache of version %d", path, kTuneFileVersion);
    }
    for (const auto& kv : loaded) g_tune[kv.first] = kv.second;
    g_tune_path = path;
    g_last_error.clear();
    return M3S_OK;
}

void m3s_batched_last_launch(m3s_launch_config* cfg) {
    if (!cfg) return;
    cfg->tile_config = g_last_tile;
    cfg->grid = g_last_grid;
    cfg->xcd_remap = -1;
    cfg->ray_margin = g_last_margin;
    cfg->lm_unroll = g_last_unroll;
}

m3s_status m3s_path_counters(int64_t* counts, int32_t reset) {
    if (!counts) return fail(M3S_ERR_NULL, "counts is NULL");
    int dev;
    DeviceInfo info;
    m3s_status s = current_device(&dev, &info);
    if (s != M3S_OK) return s;
    hipError_t e = m3s::read_path_counters(counts, reset != 0);
    if (e != hipSuccess) return hip_fail(e, "path counters");
    g_last_error.clear();
    return M3S_OK;
}

void m3s_batched_last_config(int32_t* grid, int32_t* tile_config) {
    if (grid) *grid = g_last_grid;
    if (tile_config) *tile_config = g_last_tile;
}

void m3s_clear_caches(void) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto& kv : g_graphs) hipGraphExecDestroy(kv.second);
    g_graphs.clear();
    g_tune.clear();
}

const char* m3s_status_string(m3s_status s) {
    switch (s) {
        case M3S_OK: return "ok";
        case M3S_ERR_NULL: return "required pointer is NULL";
        case M3S_ERR_SHAPE: return "invalid shape";
        case M3S_ERR_PARAM: return "invalid parameter";
        case M3S_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case M3S_ERR_HIP: return "HIP runtime error";
        case M3S_ERR_UNSUPPORTED: return "unsupported device or flag";
        default: break;
    }
    return "unknown status";
}

const char* m3s_last_error(void) { return g_last_error.c_str(); }

int32_t m3s_version(void) { return M3S_VERSION; }

}  // extern "C"
