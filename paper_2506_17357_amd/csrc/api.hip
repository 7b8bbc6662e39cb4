// Host runtime of the C ABI declared in include/tga.h: argument validation,
// workspace layout on caller-owned device memory, work-item lists, kernel
// launches, HIP-graph capture of the batched step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tga.h"
#include "kernels.hip"

using namespace tga;

namespace {

thread_local std::string g_err;
thread_local tga_move_t *g_pin = nullptr;  // pinned staging, 4 KiB per host thread
thread_local int32_t *g_pin_dev = nullptr;  // the same memory as kernels address it (null: copy instead)

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return fail(TGA_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

int pinned(void **p) {
    if (!g_pin) {
        hipError_t e = hipHostMalloc((void **)&g_pin, 4096, hipHostMallocDefault);
        if (e != hipSuccess) {
            g_pin = nullptr;
            return fail(TGA_EDEVICE, "hipHostMalloc: %s", hipGetErrorString(e));
        }
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, g_pin, 0) == hipSuccess)
            g_pin_dev = (int32_t *)dp;
        else
            (void)hipGetLastError();
    }
    *p = g_pin;
    return TGA_OK;
}

struct DevProps {
    int ok = 0, cus = 0, max_lds = 0, attr_ok = 0;
};

DevProps g_props;
std::mutex g_props_mu;

int props(DevProps *out) {
    std::lock_guard<std::mutex> lk(g_props_mu);
    if (!g_props.ok) {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&g_props.cus, hipDeviceAttributeMultiprocessorCount, dev));
        int lds = 0;
        HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        // Let the evaluation kernels use the device's full LDS for dynamic
        // shared memory (their static LDS is a few bytes).  If the runtime
        // refuses, stay within the 64 KiB every launch may use.
        const int dyn = lds - 1024;
        const void *fns[] = {(const void *)k_eval_inter<false, false>, (const void *)k_eval_inter<true, false>,
                             (const void *)k_eval_inter<false, true>, (const void *)k_eval_inter<true, true>,
                             (const void *)k_eval_batch<1>, (const void *)k_eval_batch<2>,
                             (const void *)k_eval_batch<3>, (const void *)k_eval_batch<5>,
                             (const void *)k_eval_batch<7>,
                             (const void *)k_eval_solution<false, false>, (const void *)k_eval_solution<true, false>,
                             (const void *)k_eval_solution<false, true>, (const void *)k_eval_solution<true, true>,
                             (const void *)k_eval_gran_fused<false, false>, (const void *)k_eval_gran_fused<true, false>,
                             (const void *)k_eval_gran_fused<false, true>, (const void *)k_eval_gran_fused<true, true>};
        bool ok = dyn > 65536;
        for (const void *f : fns)
            if (ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) ok = false;
        (void)hipGetLastError();  // do not leave a refused attribute as the sticky error
        g_props.attr_ok = ok;
        g_props.max_lds = ok ? dyn : std::min(lds, 65536);
        g_props.ok = 1;
    }
    *out = g_props;
    return TGA_OK;
}

// LDS per inter-route workgroup used to size the row sub-blocks: 64 KiB
// lets two workgroups share a CU.  TGA_LDS_KB overrides it (tuning).
size_t lds_budget() {
    static size_t b = [] {
        const char *e = getenv("TGA_LDS_KB");
        const long kb = (e && *e) ? atol(e) : 64;
        return (size_t)std::max(16L, std::min(160L, kb)) * 1024;
    }();
    return b;
}

constexpr int kMaxSlots = 1024;   // slots of a slot batch (served form)
constexpr int kMaxTileRows = 64;  // rows per inter-route sub-block (128 was slower on the mix)

// LDS of an inter-route workgroup with sub-blocks of h rows: the h rows and
// one halo row on each side, 16- or 32-bit.
size_t rows_lds(int np1, int h, bool w16) {
    return (size_t)(h + 2) * (w16 ? 2 * (size_t)stride16_of(np1) : 4 * (size_t)np1);
}

// Largest sub-block (at most kMaxTileRows rows) that fits the LDS budget of one
// workgroup; at least 1.
int default_tile_rows(int np1, bool w16) {
    int h = 1;
    while (h < kMaxTileRows && rows_lds(np1, h + 1, w16) <= lds_budget()) ++h;
    return h;
}

// Rows per inter-route item of the single-solution form: thin enough that a
// solution gives about 512 items (two per compute unit), at most what fits
// the LDS budget.
int plain_rows(int Q, int np1, bool w16) {
    return std::max(1, std::min(default_tile_rows(np1, w16), (Q + 511) / 512));
}

// Tuning table (tga_set_tuning): per problem kind, entries sorted by n_max;
// the first entry of the solution's kind with n <= n_max gives its rows.
std::mutex g_tune_mu;
std::vector<tga_tune_entry_t> g_tune;

void tuned_rows(int has_tw, int n, int *plain, int *item) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *plain = *item = 0;
    for (const tga_tune_entry_t &e : g_tune)
        if (e.has_tw == has_tw && n <= e.n_max) {
            *plain = e.plain_rows;
            *item = e.item_rows;
            return;
        }
}

// Inter-route items of one solution: row blocks of `rows` rows, each against
// every column slot to its right.
template <class F>
void for_each_item(int Q, int rows, F f) {
    for (int s0 = 0; s0 < Q; s0 += rows)
        f(s0, std::min(Q, s0 + rows));
}

long long count_items(int Q, int rows) {
    long long c = 0;
    for_each_item(Q, rows, [&](int, int) { ++c; });
    return c;
}

struct SolLayout {
    size_t desc, a4, b4, t4, w4, pf4, pb4, pl4, ql4, pdist, ref2slot, roff, rdist, nr_alt, roff_alt, rblk, best_key, rec,
        state, acc, items, intra, total;
    int max_items;
};

SolLayout sol_layout(int n, int R) {
    SolLayout L;
    const size_t Q = (size_t)n + R, S = Q + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.desc = take(sizeof(SolDev));
    L.a4 = take(16 * S);
    L.b4 = take(16 * S);
    L.t4 = take(16 * S);
    L.w4 = take(16 * S);
    L.pf4 = take(16 * S);
    L.pb4 = take(16 * S);
    L.pl4 = take(16 * S);
    L.ql4 = take(16 * S);
    L.pdist = take(4 * S);
    L.ref2slot = take(4 * Q);
    L.roff = take(4 * (R + 1));
    L.rdist = take(4 * std::max(R, 1));
    L.nr_alt = take(8 * S);
    L.roff_alt = take(4 * (R + 1));
    L.rblk = take(4 * (size_t)kRouteBlockWords * std::max(R, 1));
    L.best_key = take(8);
    // last record, state and accumulators back to back, so that every host
    // call reads what it needs with one copy
    L.rec = take(32 + 4 * 16 + 8 * kAccCount);
    L.state = L.rec + 32;
    L.acc = L.state + 4 * 16;
    // room for one-row items (the smallest rows per item a schedule may give)
    L.max_items = (int)Q;
    L.items = take(sizeof(InterItem) * L.max_items);
    L.intra = take(sizeof(IntraItem) * std::max(R, 1));  // at most one group per route
    L.total = off;
    return L;
}

}  // namespace

struct tga_instance {
    int32_t n, cap, has_tw;
    const int32_t *D;
    const uint16_t *D16;  // in the instance workspace; null when some distance >= 2^16
    int32_t stride16;
    const int4 *node4;
    int32_t maxD, maxE, maxL, maxS, maxDem;
    // granular neighbourhood (tga_instance_set_granular), in a caller
    // workspace: the customer-customer adjacency entries (source and
    // neighbour node, both orders) first, then the customers paired with the
    // depot (gsrc only)
    int32_t theta = 0, gnnz = 0, gcc = 0, gdep = 0;
    const int32_t *gsrc = nullptr, *gadj = nullptr;
    // pickups (tga_instance_set_pickups), borrowed; null without
    const int32_t *pick = nullptr;
    int32_t maxPick = 0;
    void *ws = nullptr;  // the instance workspace (check results, 16-bit copy of D)
};

struct tga_solution {
    tga_instance *inst;
    int32_t n, R, Q;
    SolDev h;          // host copy of the descriptor
    SolDev *d;         // device copy (1 entry)
    InterItem *items;  // device
    int nitems;
    IntraItem *intra;  // device
    int nintra;
    int tile_rows;   // rows one workgroup's LDS budget holds (batched form)
    int plain_rows;  // rows per item of the single-solution form
    int item_rows;   // rows per inter-route item of the batched form (0: the default rule)
    size_t lds;
    uint32_t version;
    int in_batch;
};

struct tga_batch {
    std::vector<tga_solution *> sols;
    SolDev *d;
    InterItem *items;
    int nitems;
    IntraItem *intra;
    int nintra;
    int *woff;      // device: inter items of XCD x = items[woff[x] .. woff[x+1]), largest first
    uint32_t *qctr; // device: per XCD {items taken, workgroups done} of the launch in flight (zero between launches)
    int *ixoff;     // device: intra-route groups of XCD x = intra[ixoff[x] .. ixoff[x+1])
    int nx;         // XCDs the items are spread over
    int32_t *done;  // per-solution converged flags gathered by tga_batch_poll
    int32_t *steps; // device: evaluation steps run (advanced by the finalize launch)
    long long *coll = nullptr;    // device: {steps, version, moves, cost} per solution (k_collect)
    long long *coll_h = nullptr;  // pinned host copy of coll
    size_t lds;
    size_t lds_intra;
    int grid_inter, grid_intra;
    tga_batch_config_t cfg;  // the schedule the plan was made for
    int max_items, max_intra;  // workspace capacity of the item lists
    hipGraphExec_t exec;
    hipGraph_t graph;
    int graph_steps;
    uint32_t graph_mask;
    hipStream_t cap_stream;  // library-owned stream used only for graph capture
    // slot batches (served form): a fixed number of slots whose members
    // change while the batch runs; sols[i] == nullptr marks an empty slot
    int slotted = 0;
    int max_sum_q = 0, max_sum_r = 0;
    char *stage_h[2] = {nullptr, nullptr};  // pinned staging of plan uploads, used in turn
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    size_t stage_bytes = 0;
    int stage_k = 0;
    long long *tick_h[2] = {nullptr, nullptr};  // pinned per-slot results of the last two ticks
    hipEvent_t tick_ev[2] = {nullptr, nullptr};
    int tick_seq[2] = {-1, -1};  // tick number whose results each buffer receives
    int ticks = 0;               // ticks launched
    hipGraphExec_t tick_exec = nullptr;
    hipGraph_t tick_graph = nullptr;
    int tick_steps = -1;
    uint32_t tick_mask = 0;
};

// ----------------------------------------------------------------- misc ----

extern "C" const char *tga_last_error(void) { return g_err.c_str(); }

extern "C" int tga_device_limits(int32_t *compute_units, int32_t *max_lds_bytes) {
    DevProps P;
    int rc = props(&P);
    if (rc) return rc;
    if (compute_units) *compute_units = P.cus;
    if (max_lds_bytes) *max_lds_bytes = P.max_lds;
    return TGA_OK;
}

// Instance workspace: 256 bytes of check results, then room for the 16-bit
// copy of D.
extern "C" size_t tga_instance_workspace_bytes(int32_t n) {
    if (n < 1 || n > TGA_MAX_Q) return 0;
    const size_t np1 = (size_t)n + 1;
    return 256 + 2 * np1 * (size_t)stride16_of((int)np1);
}

extern "C" size_t tga_solution_workspace_bytes(int32_t n, int32_t R) {
    if (n < 1 || R < 1 || (int64_t)n + R > TGA_MAX_Q) return 0;
    return sol_layout(n, R).total;
}

// ------------------------------------------------------------- instance ----

extern "C" int tga_load_instance(int32_t n, const int32_t *dist, const int32_t *node4,
                                 int32_t capacity, int32_t has_tw, void *ws, size_t ws_bytes,
                                 void *stream, tga_instance_t *out) {
    if (!out) return fail(TGA_EINVAL, "out is null");
    *out = nullptr;
    if (!dist || !node4 || !ws) return fail(TGA_EINVAL, "null device pointer");
    if (n < 1 || n > TGA_MAX_Q - 1) return fail(TGA_ERANGE, "n = %d outside [1, %d]", n, TGA_MAX_Q - 1);
    if (capacity < 0 || capacity >= (1 << 30)) return fail(TGA_ERANGE, "capacity %d", capacity);
    if (has_tw != 0 && has_tw != 1) return fail(TGA_EINVAL, "has_tw must be 0 or 1");
    if (ws_bytes < tga_instance_workspace_bytes(n)) return fail(TGA_ENOMEM, "instance workspace too small");
    if (((uintptr_t)node4) & 15) return fail(TGA_EINVAL, "node4 must be 16-byte aligned");
    if (((uintptr_t)ws) & 255) return fail(TGA_EINVAL, "workspace must be 256-byte aligned");
    DevProps P;
    int rc = props(&P);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int np1 = n + 1;
    int32_t *chk = (int32_t *)ws;
    k_zero_i32<<<1, 64, 0, st>>>(chk, 8);
    const int tiles = (np1 + 31) / 32;
    k_check_dist<<<dim3(tiles, tiles), 256, 0, st>>>(dist, np1, chk);
    k_check_nodes<<<(np1 + 255) / 256, 256, 0, st>>>((const int4 *)node4, np1, has_tw, chk);
    HIPCHK(hipGetLastError());
    void *pin;
    if ((rc = pinned(&pin))) return rc;
    HIPCHK(hipMemcpyAsync(pin, chk, 32, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int32_t r[8];
    memcpy(r, pin, 32);
    if (r[0] & 1) return fail(TGA_EINVAL, "distance outside [0, 2^24)");
    if (r[0] & 2) return fail(TGA_EINVAL, "distance matrix is not symmetric");
    if (r[0] & 4) return fail(TGA_EINVAL, "distance matrix has a nonzero diagonal");
    if (r[0] & 8) return fail(TGA_EINVAL, "bad node data (negative, e > l, or depot demand/service != 0)");
    const int64_t maxD = r[1], maxE = r[2], maxL = r[3], maxS = r[4], maxDem = r[5];
    if ((int64_t)n * maxDem >= (1 << 30)) return fail(TGA_ERANGE, "total demand may exceed 2^30");
    if (has_tw && (int64_t)np1 * (maxS + maxD) + maxL + maxE >= (1 << 28))
        return fail(TGA_ERANGE, "route durations may exceed 2^28");
    const int stride16 = stride16_of(np1);
    uint16_t *d16 = nullptr;
    if (maxD < 65536) {  // every distance fits 16 bits: keep a packed copy for the inter-route kernels
        d16 = (uint16_t *)((char *)ws + 256);
        k_pack16<<<dim3((stride16 + 255) / 256, np1), 256, 0, st>>>(dist, np1, stride16, d16);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    }
    tga_instance *I = new tga_instance;
    I->n = n;
    I->cap = capacity;
    I->has_tw = has_tw;
    I->D = dist;
    I->D16 = d16;
    I->stride16 = stride16;
    I->node4 = (const int4 *)node4;
    I->maxD = (int32_t)maxD;
    I->maxE = (int32_t)maxE;
    I->maxL = (int32_t)maxL;
    I->maxS = (int32_t)maxS;
    I->maxDem = (int32_t)maxDem;
    I->ws = ws;
    *out = I;
    return TGA_OK;
}

extern "C" size_t tga_granular_workspace_bytes(int32_t n, int32_t theta) {
    if (n < 1 || n > TGA_MAX_Q - 1 || theta < 1 || theta > n || theta > kKnnMax) return 0;
    const size_t np1 = (size_t)n + 1;
    // theta nearest of every node, then source and neighbour of up to
    // 2 theta (n+1) adjacency entries
    return align_up(4 * np1 * theta, 256) + 2 * align_up(4 * 2 * np1 * (size_t)theta, 256);
}

extern "C" int tga_instance_set_granular(tga_instance_t inst, int32_t theta, void *ws, size_t ws_bytes,
                                         void *stream) {
    if (!inst || !ws) return fail(TGA_EINVAL, "null argument");
    const int n = inst->n, np1 = n + 1;
    const size_t need = tga_granular_workspace_bytes(n, theta);
    if (!need) return fail(TGA_ERANGE, "theta = %d outside [1, min(n, %d)]", theta, kKnnMax);
    if (ws_bytes < need) return fail(TGA_ENOMEM, "granular workspace %zu < %zu", ws_bytes, need);
    if (((uintptr_t)ws) & 255) return fail(TGA_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    int32_t *nn = (int32_t *)ws;
    k_knn<<<np1, 256, 0, st>>>(inst->D, np1, theta, nn);
    HIPCHK(hipGetLastError());
    std::vector<int32_t> h((size_t)np1 * theta);
    HIPCHK(hipMemcpyAsync(h.data(), nn, 4 * h.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // symmetric closure: j is listed under i when either is among the other's
    // theta nearest; only the rows of customers are kept (the depot's pairs
    // are walked from its customers)
    std::vector<std::vector<int32_t>> adj(np1);
    for (int i = 0; i < np1; ++i)
        for (int k = 0; k < theta; ++k) {
            const int j = h[(size_t)i * theta + k];
            if (j < 0 || j > n || j == i) return fail(TGA_EDEVICE, "neighbour list of node %d is corrupt", i);
            adj[i].push_back(j);
            adj[j].push_back(i);
        }
    std::vector<int32_t> src, dst, dep;
    for (int i = 1; i < np1; ++i) {
        std::sort(adj[i].begin(), adj[i].end());
        adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
        for (int j : adj[i]) {
            if (j == 0) {
                dep.push_back(i);
                continue;
            }
            src.push_back(i);
            dst.push_back(j);
        }
    }
    const int32_t gcc = (int32_t)src.size(), gdep = (int32_t)dep.size();
    src.insert(src.end(), dep.begin(), dep.end());
    dst.resize(src.size(), 0);
    int32_t *gsrc = (int32_t *)((char *)ws + align_up(4 * (size_t)np1 * theta, 256));
    int32_t *gadj = (int32_t *)((char *)gsrc + align_up(4 * 2 * (size_t)np1 * theta, 256));
    if (!src.empty()) {
        HIPCHK(hipMemcpyAsync(gsrc, src.data(), 4 * src.size(), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(gadj, dst.data(), 4 * dst.size(), hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    inst->theta = theta;
    inst->gnnz = (int32_t)src.size();
    inst->gcc = gcc;
    inst->gdep = gdep;
    inst->gsrc = gsrc;
    inst->gadj = gadj;
    return TGA_OK;
}

extern "C" int32_t tga_instance_granular_pairs(tga_instance_t inst) { return inst ? inst->gnnz : 0; }

extern "C" int tga_instance_set_pickups(tga_instance_t inst, const int32_t *pickup, void *stream) {
    if (!inst || !pickup) return fail(TGA_EINVAL, "null argument");
    const int np1 = inst->n + 1;
    hipStream_t st = (hipStream_t)stream;
    int32_t chk[2] = {0, 0};
    // the check results go through the instance workspace's check area (its first 256 bytes)
    int32_t *dchk = (int32_t *)((char *)inst->ws + 64);
    k_zero_i32<<<1, 64, 0, st>>>(dchk, 2);
    k_check_pick<<<(np1 + 255) / 256, 256, 0, st>>>(pickup, np1, dchk);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(chk, dchk, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (chk[0] & 1) return fail(TGA_EINVAL, "pickups must be >= 0, with 0 at the depot");
    const int64_t maxP = chk[1];
    if ((int64_t)inst->n * std::max<int64_t>(maxP, inst->maxDem) * 2 >= (1 << 30))
        return fail(TGA_ERANGE, "loads with pickups may exceed 2^30");
    inst->pick = pickup;
    inst->maxPick = (int32_t)maxP;
    return TGA_OK;
}

extern "C" int32_t tga_instance_dist_bytes(tga_instance_t inst) {
    if (!inst) return 0;
    return inst->D16 ? 2 : 4;
}

extern "C" int tga_free_instance(tga_instance_t inst) {
    delete inst;
    return TGA_OK;
}

// ------------------------------------------------------------- solution ----

static int check_partition(int n, int R, const int32_t *offsets, const int32_t *customers);

// Intra-route items: groups of consecutive routes whose customers typically
// fill about 48 of a wavefront's 64 lanes (the kernel falls back to one route
// at a time when a group has grown beyond what its wavefront can stage).
static void push_intra_groups(int n, int R, int sol_index, std::vector<IntraItem> &intra) {
    const int avgL = std::max(1, n / std::max(1, R));
    const int G = std::max(1, std::min(kIntraMaxGroup, 48 / (avgL + 1)));
    for (int r = 0; r < R; r += G) intra.push_back(IntraItem{sol_index, r, std::min(R, r + G), 0});
}

static void build_plain_items(tga_solution *S, std::vector<InterItem> &items,
                              std::vector<IntraItem> &intra, int sol_index) {
    for_each_item(S->Q, S->plain_rows,
                  [&](int s0, int s1) { items.push_back(InterItem{sol_index, s0, s1, 0}); });
    push_intra_groups(S->n, S->R, sol_index, intra);
}

// Argument checks shared by every way of setting up a solution.
static int check_solution_args(tga_instance_t inst, int32_t R, const int32_t *offsets,
                               const int32_t *customers) {
    if (!inst || !offsets || !customers) return fail(TGA_EINVAL, "null argument");
    const int n = inst->n;
    if (R < 1) return fail(TGA_ERANGE, "R = %d < 1", R);
    if ((int64_t)n + R > TGA_MAX_Q) return fail(TGA_ERANGE, "n + R = %lld > %d", (long long)n + R, TGA_MAX_Q);
    if ((int64_t)(n + R + 1) * inst->maxD >= (1 << 30)) return fail(TGA_ERANGE, "total distance may exceed 2^30");
    return check_partition(n, R, offsets, customers);
}

// Lay a solution out in the workspace at `ws` (checked by the caller: large
// enough, 256-byte aligned), upload its routes and build its attributes.
// Fills *S; synchronises `st`.  Allocates no device or pinned memory.
static int solution_init(tga_solution *S, tga_instance_t inst, int32_t R, const int32_t *offsets,
                         const int32_t *customers, void *ws, hipStream_t st) {
    const int n = inst->n;
    const SolLayout L = sol_layout(n, R);
    DevProps P;
    int rc = props(&P);
    if (rc) return rc;
    const int Q = n + R, np1 = n + 1;
    S->inst = inst;
    S->n = n;
    S->R = R;
    S->Q = Q;
    const bool w16 = inst->D16 != nullptr;
    S->tile_rows = default_tile_rows(np1, w16);
    int t_plain, t_item;
    tuned_rows(inst->has_tw, n, &t_plain, &t_item);
    S->plain_rows = t_plain > 0 ? std::min(t_plain, S->tile_rows) : plain_rows(Q, np1, w16);
    S->item_rows = t_item;
    S->lds = rows_lds(np1, S->plain_rows, w16);
    if (S->lds > (size_t)P.max_lds)
        return fail(TGA_ERANGE, "n = %d needs %zu bytes of LDS per workgroup (device: %d)", n,
                    rows_lds(np1, 1, w16), P.max_lds);
    char *base = (char *)ws;
    SolDev &h = S->h;
    memset(&h, 0, sizeof h);
    h.D = inst->D;
    h.D16 = inst->D16;
    h.stride16 = inst->stride16;
    h.node4 = inst->node4;
    h.n = n;
    h.np1 = np1;
    h.cap = inst->cap;
    h.has_tw = inst->has_tw;
    h.R = R;
    h.Q = Q;
    h.tile_rows = S->plain_rows;
    h.a4 = (int4 *)(base + L.a4);
    h.b4 = (int4 *)(base + L.b4);
    h.t4 = (int4 *)(base + L.t4);
    h.w4 = (int4 *)(base + L.w4);
    h.pf4 = (int4 *)(base + L.pf4);
    h.pb4 = (int4 *)(base + L.pb4);
    h.pl4 = (int4 *)(base + L.pl4);
    h.ql4 = (int4 *)(base + L.ql4);
    h.pick = inst->pick;
    h.pd = inst->pick != nullptr;
    h.pdist = (int32_t *)(base + L.pdist);
    h.ref2slot = (int32_t *)(base + L.ref2slot);
    h.roff = (int32_t *)(base + L.roff);
    h.rdist = (int32_t *)(base + L.rdist);
    h.nr_alt = (int2 *)(base + L.nr_alt);
    h.roff_alt = (int32_t *)(base + L.roff_alt);
    h.rblk = (int32_t *)(base + L.rblk);
    h.best_key = (unsigned long long *)(base + L.best_key);
    h.rec = (int32_t *)(base + L.rec);
    h.state = (int32_t *)(base + L.state);
    h.acc = (long long *)(base + L.acc);
    S->d = (SolDev *)(base + L.desc);
    S->items = (InterItem *)(base + L.items);
    S->intra = (IntraItem *)(base + L.intra);

    // host-side layout: slots route-major with the start depot first
    std::vector<int2> nr(Q + 1);
    std::vector<int32_t> roff(R + 1);
    int s = 0;
    for (int r = 0; r < R; ++r) {
        roff[r] = s;
        nr[s++] = make_int2(0, r);
        for (int i = offsets[r]; i < offsets[r + 1]; ++i) nr[s++] = make_int2(customers[i], r);
    }
    roff[R] = s;
    nr[Q] = make_int2(0, R);
    std::vector<InterItem> items;
    std::vector<IntraItem> intra;
    build_plain_items(S, items, intra, 0);
    S->nitems = (int)items.size();
    S->nintra = (int)intra.size();
    if (S->nitems > L.max_items) return fail(TGA_ERANGE, "too many work items");
    std::vector<int32_t> state(16, 0);
    std::vector<long long> acc(kAccCount, 0);
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(S->d, &h, sizeof h);
    if (e == hipSuccess) e = up(h.nr_alt, nr.data(), sizeof(int2) * (Q + 1));
    if (e == hipSuccess) e = up(h.roff_alt, roff.data(), sizeof(int32_t) * (R + 1));
    if (e == hipSuccess) e = up(h.state, state.data(), sizeof(int32_t) * 16);
    if (e == hipSuccess) e = up(h.acc, acc.data(), sizeof(long long) * kAccCount);
    if (e == hipSuccess) e = up(S->items, items.data(), sizeof(InterItem) * items.size());
    if (e == hipSuccess) e = up(S->intra, intra.data(), sizeof(IntraItem) * intra.size());
    if (e == hipSuccess) {
        k_route_blocks_clear<<<(R + 255) / 256, 256, 0, st>>>(h.rblk, R);
        k_build<<<1, kApplyThreads, 0, st>>>(S->d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(TGA_EDEVICE, "set_solution: %s", hipGetErrorString(e));
    return TGA_OK;
}

extern "C" int tga_set_tuning(const tga_tune_entry_t *entries, int32_t count) {
    if (count < 0 || (count > 0 && !entries)) return fail(TGA_EINVAL, "bad entry list");
    std::vector<tga_tune_entry_t> t(entries, entries + count);
    for (const tga_tune_entry_t &e : t)
        if ((e.has_tw != 0 && e.has_tw != 1) || e.n_max < 1 || e.plain_rows < 0 || e.item_rows < 0 ||
            e.plain_rows > TGA_MAX_Q || e.item_rows > TGA_MAX_Q)
            return fail(TGA_EINVAL, "bad tuning entry (has_tw %d, n_max %d, rows %d / %d)", e.has_tw, e.n_max,
                        e.plain_rows, e.item_rows);
    std::stable_sort(t.begin(), t.end(), [](const tga_tune_entry_t &a, const tga_tune_entry_t &b) {
        return a.has_tw != b.has_tw ? a.has_tw < b.has_tw : a.n_max < b.n_max;
    });
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.swap(t);
    return TGA_OK;
}

extern "C" int tga_solution_set_rows(tga_solution_t sol, int32_t plain_rows_, int32_t item_rows, void *stream) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    if (sol->in_batch) return fail(TGA_EINVAL, "solution belongs to a batch");
    if (plain_rows_ < 0 || item_rows < 0 || plain_rows_ > TGA_MAX_Q || item_rows > TGA_MAX_Q)
        return fail(TGA_EINVAL, "rows out of range");
    const bool w16 = sol->h.D16 != nullptr;
    int t_plain, t_item;
    tuned_rows(sol->inst->has_tw, sol->n, &t_plain, &t_item);
    if (plain_rows_ == 0) plain_rows_ = t_plain;
    sol->plain_rows = plain_rows_ > 0 ? std::min(plain_rows_, sol->tile_rows) : plain_rows(sol->Q, sol->n + 1, w16);
    sol->item_rows = item_rows > 0 ? item_rows : t_item;
    sol->lds = rows_lds(sol->n + 1, sol->plain_rows, w16);
    sol->h.tile_rows = sol->plain_rows;
    std::vector<InterItem> items;
    std::vector<IntraItem> intra;
    build_plain_items(sol, items, intra, 0);
    sol->nitems = (int)items.size();
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(sol->items, items.data(), sizeof(InterItem) * items.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(sol->d, &sol->h, sizeof(SolDev), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return TGA_OK;
}

extern "C" int tga_solution_get_rows(tga_solution_t sol, int32_t *plain_rows_, int32_t *item_rows) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    if (plain_rows_) *plain_rows_ = sol->plain_rows;
    if (item_rows) *item_rows = sol->item_rows;
    return TGA_OK;
}

extern "C" int tga_set_solution(tga_instance_t inst, int32_t R, const int32_t *offsets,
                                const int32_t *customers, void *ws, size_t ws_bytes, void *stream,
                                tga_solution_t *out) {
    if (!out) return fail(TGA_EINVAL, "out is null");
    *out = nullptr;
    if (!ws) return fail(TGA_EINVAL, "null argument");
    int rc = check_solution_args(inst, R, offsets, customers);
    if (rc) return rc;
    const SolLayout L = sol_layout(inst->n, R);
    if (ws_bytes < L.total) return fail(TGA_ENOMEM, "solution workspace %zu < %zu", ws_bytes, L.total);
    if (((uintptr_t)ws) & 255) return fail(TGA_EINVAL, "workspace must be 256-byte aligned");
    tga_solution *S = new tga_solution();
    if ((rc = solution_init(S, inst, R, offsets, customers, ws, (hipStream_t)stream))) {
        delete S;
        return rc;
    }
    *out = S;
    return TGA_OK;
}

static int check_partition(int n, int R, const int32_t *offsets, const int32_t *customers) {
    if (offsets[0] != 0 || offsets[R] != n) return fail(TGA_EINVAL, "offsets must start at 0 and end at n");
    for (int r = 0; r < R; ++r)
        if (offsets[r + 1] < offsets[r]) return fail(TGA_EINVAL, "offsets decrease at route %d", r);
    std::vector<char> seen(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        const int c = customers[i];
        if (c < 1 || c > n || seen[c]) return fail(TGA_EINVAL, "customers is not a permutation of 1..n (at %d)", i);
        seen[c] = 1;
    }
    return TGA_OK;
}

extern "C" int tga_solution_reload(tga_solution_t sol, const int32_t *offsets, const int32_t *customers,
                                   void *stream) {
    if (!sol || !offsets || !customers) return fail(TGA_EINVAL, "null argument");
    const int n = sol->n, R = sol->R, Q = sol->Q;
    int rc = check_partition(n, R, offsets, customers);
    if (rc) return rc;
    std::vector<int2> nr(Q + 1);
    std::vector<int32_t> roff(R + 1);
    int s = 0;
    for (int r = 0; r < R; ++r) {
        roff[r] = s;
        nr[s++] = make_int2(0, r);
        for (int i = offsets[r]; i < offsets[r + 1]; ++i) nr[s++] = make_int2(customers[i], r);
    }
    roff[R] = s;
    nr[Q] = make_int2(0, R);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(sol->h.nr_alt, nr.data(), sizeof(int2) * (Q + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(sol->h.roff_alt, roff.data(), sizeof(int32_t) * (R + 1), hipMemcpyHostToDevice, st));
    k_reset_state<<<1, 64, 0, st>>>(sol->d, 1, 0);
    k_route_blocks_clear<<<(R + 255) / 256, 256, 0, st>>>(sol->h.rblk, R);  // start cold, as a new solution
    k_build<<<1, kApplyThreads, 0, st>>>(sol->d);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    sol->version = 0;
    return TGA_OK;
}

extern "C" int tga_solution_begin(tga_solution_t sol, int32_t max_steps, void *stream) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    if (max_steps < 0) return fail(TGA_EINVAL, "max_steps < 0");
    k_reset_state<<<1, 64, 0, (hipStream_t)stream>>>(sol->d, 1, max_steps);
    HIPCHK(hipGetLastError());
    return TGA_OK;
}

extern "C" int tga_free_solution(tga_solution_t sol) {
    delete sol;
    return TGA_OK;
}

extern "C" uint32_t tga_solution_version(tga_solution_t sol) { return sol ? sol->version : 0; }

// Granular mode: the inter-route moves of the granular pairs (one launch of
// k_eval_gran), the intra-route ones complete (k_eval_intra).
static void launch_eval_gran(const tga_instance *I, const SolDev *d, int R, const IntraItem *intra, int nintra,
                             int has_tw, uint32_t op_mask, int32_t *dd, uint8_t *df, hipStream_t st) {
    const bool dump = dd != nullptr;
    const long long work = I->gcc + (long long)I->gdep * R;
    if ((op_mask & 7) && work > 0 && (op_mask & (2 | 8 | 16)) && nintra > 0) {
        // both kinds in one launch: the intra-route groups first, then the pairs
        const int grid = nintra + (int)((work + kInterThreads - 1) / kInterThreads);
        const size_t l = (size_t)kInterWaves * kIntraRegionBytes;
        const int a = I->gcc, b = I->gdep;
        if (has_tw) {
            if (dump)
                k_eval_gran_fused<true, true><<<grid, kInterThreads, l, st>>>(d, I->gsrc, I->gadj, a, b, intra, nintra,
                                                                             op_mask, dd, df);
            else
                k_eval_gran_fused<true, false><<<grid, kInterThreads, l, st>>>(d, I->gsrc, I->gadj, a, b, intra,
                                                                              nintra, op_mask, dd, df);
        } else {
            if (dump)
                k_eval_gran_fused<false, true><<<grid, kInterThreads, l, st>>>(d, I->gsrc, I->gadj, a, b, intra,
                                                                              nintra, op_mask, dd, df);
            else
                k_eval_gran_fused<false, false><<<grid, kInterThreads, l, st>>>(d, I->gsrc, I->gadj, a, b, intra,
                                                                               nintra, op_mask, dd, df);
        }
        return;
    }
    if ((op_mask & 7) && work > 0) {
        const int grid = (int)((work + 255) / 256);
        const int a = I->gcc, b = I->gdep;
        if (has_tw) {
            if (dump)
                k_eval_gran<true, true><<<grid, 256, 0, st>>>(d, I->gsrc, I->gadj, a, b, op_mask, dd, df);
            else
                k_eval_gran<true, false><<<grid, 256, 0, st>>>(d, I->gsrc, I->gadj, a, b, op_mask, dd, df);
        } else {
            if (dump)
                k_eval_gran<false, true><<<grid, 256, 0, st>>>(d, I->gsrc, I->gadj, a, b, op_mask, dd, df);
            else
                k_eval_gran<false, false><<<grid, 256, 0, st>>>(d, I->gsrc, I->gadj, a, b, op_mask, dd, df);
        }
    }
    if ((op_mask & (2 | 8 | 16)) && nintra > 0) {
        const size_t ilds = (size_t)kInterWaves * kIntraRegionBytes;
        if (has_tw) {
            if (dump)
                k_eval_intra<true, true><<<nintra, kInterThreads, ilds, st>>>(d, intra, nintra, op_mask, dd, df);
            else
                k_eval_intra<true, false><<<nintra, kInterThreads, ilds, st>>>(d, intra, nintra, op_mask, dd, df);
        } else {
            if (dump)
                k_eval_intra<false, true><<<nintra, kInterThreads, ilds, st>>>(d, intra, nintra, op_mask, dd, df);
            else
                k_eval_intra<false, false><<<nintra, kInterThreads, ilds, st>>>(d, intra, nintra, op_mask, dd, df);
        }
    }
}

static void launch_eval(const SolDev *d, const InterItem *items, int nitems, const IntraItem *intra,
                        int nintra, int has_tw, uint32_t op_mask, size_t lds, int grid_inter,
                        int32_t *dd, uint8_t *df, hipStream_t st) {
    const bool dump = dd != nullptr;
    if ((op_mask & 7) && nitems > 0 && (op_mask & (2 | 8 | 16)) && nintra > 0) {
        // both kinds in one launch: one workgroup per intra-route group first
        // (their walks are the launch's longest chains), then the inter-route
        // workgroups
        const int ninter = std::max(1, std::min(nitems, grid_inter));
        const int nbintra = nintra;
        const int grid = nbintra + ninter;
        const size_t l = std::max(lds, (size_t)kInterWaves * kIntraRegionBytes);
        if (has_tw) {
            if (dump)
                k_eval_solution<true, true><<<grid, kInterThreads, l, st>>>(d, items, nitems, intra, nintra, nbintra,
                                                                            op_mask, dd, df);
            else
                k_eval_solution<true, false><<<grid, kInterThreads, l, st>>>(d, items, nitems, intra, nintra, nbintra,
                                                                             op_mask, dd, df);
        } else {
            if (dump)
                k_eval_solution<false, true><<<grid, kInterThreads, l, st>>>(d, items, nitems, intra, nintra, nbintra,
                                                                             op_mask, dd, df);
            else
                k_eval_solution<false, false><<<grid, kInterThreads, l, st>>>(d, items, nitems, intra, nintra, nbintra,
                                                                              op_mask, dd, df);
        }
        return;
    }
    if ((op_mask & 7) && nitems > 0) {
        const int grid = std::max(1, std::min(nitems, grid_inter));
        if (has_tw) {
            if (dump)
                k_eval_inter<true, true><<<grid, kInterThreads, lds, st>>>(d, items, nitems, op_mask, dd, df);
            else
                k_eval_inter<true, false><<<grid, kInterThreads, lds, st>>>(d, items, nitems, op_mask, dd, df);
        } else {
            if (dump)
                k_eval_inter<false, true><<<grid, kInterThreads, lds, st>>>(d, items, nitems, op_mask, dd, df);
            else
                k_eval_inter<false, false><<<grid, kInterThreads, lds, st>>>(d, items, nitems, op_mask, dd, df);
        }
    }
    if ((op_mask & (2 | 8 | 16)) && nintra > 0) {
        const int grid = nintra;  // one workgroup per group: every walk has a compute unit to itself
        const size_t ilds = (size_t)kInterWaves * kIntraRegionBytes;
        if (has_tw) {
            if (dump)
                k_eval_intra<true, true><<<grid, kInterThreads, ilds, st>>>(d, intra, nintra, op_mask, dd, df);
            else
                k_eval_intra<true, false><<<grid, kInterThreads, ilds, st>>>(d, intra, nintra, op_mask, dd, df);
        } else {
            if (dump)
                k_eval_intra<false, true><<<grid, kInterThreads, ilds, st>>>(d, intra, nintra, op_mask, dd, df);
            else
                k_eval_intra<false, false><<<grid, kInterThreads, ilds, st>>>(d, intra, nintra, op_mask, dd, df);
        }
    }
}

static void to_move(const int32_t *rec, tga_move_t *m) {
    m->op = rec[0];
    m->k = rec[1];
    m->a = rec[2];
    m->b = rec[3];
    m->delta = rec[4];
    m->feas = (uint32_t)rec[5];
    m->id = (uint32_t)rec[6];
    m->version = (uint32_t)rec[7];
}

// One evaluation of a solution whose workspace is set up: evaluation launch,
// record-mode finalize, and one copy of the record and state[0..3] into
// `host` (48 bytes; pinned or pageable).
// Penalised mode: inter-route pairs (16 x 16 tiles on and above the
// diagonal) and intra-route walks (one thread per slot).
template <bool TW, bool PD>
static void launch_eval_gen(const tga_solution *sol, uint32_t op_mask, int32_t *dd, uint8_t *df, hipStream_t st) {
    const bool dump = dd != nullptr;
    if (op_mask & (7 | TGA_OP_VARIANTS)) {
        const int tiles = (sol->Q + 15) / 16, grid = tiles * (tiles + 1) / 2;
        if (dump) k_eval_pen_pairs<TW, PD, true><<<grid, 256, 0, st>>>(sol->d, tiles, op_mask, dd, df);
        else k_eval_pen_pairs<TW, PD, false><<<grid, 256, 0, st>>>(sol->d, tiles, op_mask, dd, df);
    }
    if (op_mask & (2 | 8 | 16)) {
        const int grid = (7 * sol->Q + 255) / 256;  // seven walks per slot
        if (dump) k_eval_pen_intra<TW, PD, true><<<grid, 256, 0, st>>>(sol->d, op_mask, dd, df);
        else k_eval_pen_intra<TW, PD, false><<<grid, 256, 0, st>>>(sol->d, op_mask, dd, df);
    }
}

// General path (penalised mode or pickups): gathers per pair and per walk,
// every attribute of a new route concatenated from the stored summaries.
static void launch_eval_pen(const tga_solution *sol, uint32_t op_mask, int32_t *dd, uint8_t *df, hipStream_t st) {
    const bool tw = sol->h.has_tw, pd = sol->h.pd;
    if (tw && pd) launch_eval_gen<true, true>(sol, op_mask, dd, df, st);
    else if (tw) launch_eval_gen<true, false>(sol, op_mask, dd, df, st);
    else if (pd) launch_eval_gen<false, true>(sol, op_mask, dd, df, st);
    else launch_eval_gen<false, false>(sol, op_mask, dd, df, st);
}

// Launch one evaluation of a solution (penalised, granular or full
// neighbourhood).
static void launch_solution_eval(tga_solution *sol, uint32_t op_mask, int32_t *dd, uint8_t *df, hipStream_t st) {
    if (sol->h.pen || sol->h.pd || sol->h.gen)
        launch_eval_pen(sol, op_mask, dd, df, st);
    else if (op_mask & TGA_OP_GRANULAR)
        launch_eval_gran(sol->inst, sol->d, sol->R, sol->intra, sol->nintra, sol->h.has_tw, op_mask, dd, df, st);
    else
        launch_eval(sol->d, sol->items, sol->nitems, sol->intra, sol->nintra, sol->h.has_tw, op_mask, sol->lds,
                    sol->nitems, dd, df, st);
}

// Operator mask of a single-solution call: the five operators plus the
// granular modifier (only once the instance has its granular pairs).
static int check_mask(const tga_solution *sol, uint32_t op_mask) {
    if (op_mask & ~(TGA_OP_ALL | TGA_OP_VARIANTS | TGA_OP_GRANULAR | TGA_OP_MULTI))
        return fail(TGA_EINVAL, "unknown operator bits 0x%x", op_mask);
    if (op_mask & TGA_OP_VARIANTS) {
        if (!(sol->h.pen || sol->h.pd || sol->h.gen))
            return fail(TGA_EINVAL, "operator variants need the general path (tga_solution_set_general)");
        if (sol->Q > TGA_MAX_Q_VARIANTS)
            return fail(TGA_ERANGE, "operator variants need n + R <= %d (move ids below 2^32)", TGA_MAX_Q_VARIANTS);
    }
    if ((op_mask & TGA_OP_MULTI) && !sol->h.pairkey)
        return fail(TGA_EINVAL, "TGA_OP_MULTI before tga_solution_set_multi");
    if ((op_mask & TGA_OP_GRANULAR) && !sol->inst->gnnz)
        return fail(TGA_EINVAL, "TGA_OP_GRANULAR before tga_instance_set_granular");
    if ((op_mask & TGA_OP_GRANULAR) && (sol->h.pen || sol->h.pd || sol->h.gen))
        return fail(TGA_EINVAL, "TGA_OP_GRANULAR on the general path (penalties, pickups, variants) is not supported");
    return TGA_OK;
}

extern "C" int tga_solution_set_penalty(tga_solution_t sol, int32_t w_load, int32_t w_tw, void *stream) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    if (sol->in_batch) return fail(TGA_EINVAL, "solution belongs to a batch");
    const tga_instance *I = sol->inst;
    const bool pen = w_load >= 0;
    if (pen) {
        if (w_tw < 0) return fail(TGA_EINVAL, "w_tw must be >= 0 with w_load >= 0");
        if (!I->has_tw && w_tw != 0) return fail(TGA_EINVAL, "w_tw must be 0 without time windows");
        // every score and summary must stay exact in int32
        const double np1 = (double)I->n + 1;
        const double tb = I->has_tw ? np1 * ((double)I->maxS + I->maxD + I->maxE) + I->maxL : 0.0;
        const double bound = 2.0 * w_tw * tb + 2.0 * w_load * (double)I->n * std::max(I->maxDem, I->maxPick) +
                             4.0 * ((double)sol->Q + 1) * I->maxD;
        if (tb >= (double)(1 << 28) || bound >= (double)(1 << 29))
            return fail(TGA_ERANGE, "penalty weights (%d, %d) could take a score beyond 2^29", w_load, w_tw);
    }
    sol->h.pen = pen ? 1 : 0;
    sol->h.wL = pen ? w_load : 0;
    sol->h.wT = pen ? w_tw : 0;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(sol->d, &sol->h, sizeof(SolDev), hipMemcpyHostToDevice, st));
    k_pen_init<<<1, kApplyThreads, 0, st>>>(sol->d);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return TGA_OK;
}

extern "C" int tga_solution_set_general(tga_solution_t sol, int32_t on, void *stream) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    if (sol->in_batch) return fail(TGA_EINVAL, "solution belongs to a batch");
    if (on != 0 && on != 1) return fail(TGA_EINVAL, "on must be 0 or 1");
    sol->h.gen = on;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(sol->d, &sol->h, sizeof(SolDev), hipMemcpyHostToDevice, st));
    k_pen_init<<<1, kApplyThreads, 0, st>>>(sol->d);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return TGA_OK;
}

extern "C" int tga_solution_violations(tga_solution_t sol, int64_t *load_excess, int64_t *time_warp, void *stream) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    if (!(sol->h.pen || sol->h.pd || sol->h.gen)) return fail(TGA_EINVAL, "the solution is not on the general path");
    hipStream_t st = (hipStream_t)stream;
    long long v[2];
    HIPCHK(hipMemcpyAsync(v, sol->h.acc + kAccLoadExcess, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (load_excess) *load_excess = v[0];
    if (time_warp) *time_warp = v[1];
    return TGA_OK;
}

// `host_pinned`: `host` is this thread's pinned buffer, which the finalize
// kernel writes directly (through its device address); otherwise (pageable
// memory, or no device address) the record is copied after it.
static int eval_record(tga_solution *sol, uint32_t op_mask, tga_move_t *best, int32_t *dump_delta,
                       uint8_t *dump_feas, hipStream_t st, int32_t *host, bool host_pinned) {
    int32_t *dev_view = host_pinned ? g_pin_dev : nullptr;  // where the kernel may write `host`
    launch_solution_eval(sol, op_mask, dump_delta, dump_feas, st);
    k_finalize<<<1, kApplyThreads, 0, st>>>(sol->d, kModeRecord, op_mask, nullptr, dev_view);
    HIPCHK(hipGetLastError());
    if (!dev_view)
        HIPCHK(hipMemcpyAsync(host, sol->h.rec, 32 + 16, hipMemcpyDeviceToHost, st));  // record, state[0..3]
    HIPCHK(hipStreamSynchronize(st));
    if (host[8 + kStStatus] == 1) {
        memset(best, 0, sizeof *best);
        best->version = sol->version;
        return TGA_ENOMOVE;
    }
    to_move(host, best);
    best->version = sol->version;
    return TGA_OK;
}

extern "C" int tga_eval_neighborhood(tga_solution_t sol, uint32_t op_mask, tga_move_t *best,
                                     int32_t *dump_delta, uint8_t *dump_feas, void *stream) {
    if (!sol || !best) return fail(TGA_EINVAL, "null argument");
    if ((dump_delta == nullptr) != (dump_feas == nullptr))
        return fail(TGA_EINVAL, "dump_delta and dump_feas must both be set or both be null");
    if (sol->in_batch) return fail(TGA_EINVAL, "solution belongs to a batch");
    int rc = check_mask(sol, op_mask);
    if (rc) return rc;
    DevProps P;
    if ((rc = props(&P))) return rc;
    void *pin;
    if ((rc = pinned(&pin))) return rc;
    if (op_mask & TGA_OP_MULTI) {  // the per-route-pair table starts empty
        const size_t RR = (size_t)sol->R * sol->R;
        k_fill_u64<<<(int)std::min<size_t>((RR + 255) / 256, 1024), 256, 0, (hipStream_t)stream>>>(sol->h.pairkey, RR);
        HIPCHK(hipGetLastError());
    }
    return eval_record(sol, op_mask, best, dump_delta, dump_feas, (hipStream_t)stream, (int32_t *)pin, true);
}

extern "C" size_t tga_multi_workspace_bytes(int32_t R) {
    if (R < 1) return 0;
    return align_up((size_t)R * R * 8, 256) + align_up((size_t)(1 + 2 * R) * 4, 256);
}

extern "C" int tga_solution_set_multi(tga_solution_t sol, void *ws, size_t ws_bytes, void *stream) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    if (sol->in_batch) return fail(TGA_EINVAL, "solution belongs to a batch");
    hipStream_t st = (hipStream_t)stream;
    if (!ws) {
        sol->h.pairkey = nullptr;
        sol->h.msel = nullptr;
    } else {
        if (sol->R > kMultiMaxR) return fail(TGA_ERANGE, "multi-move needs R <= %d", kMultiMaxR);
        if (ws_bytes < tga_multi_workspace_bytes(sol->R))
            return fail(TGA_ENOMEM, "multi-move workspace %zu < %zu", ws_bytes, tga_multi_workspace_bytes(sol->R));
        if (((uintptr_t)ws) & 255) return fail(TGA_EINVAL, "workspace must be 256-byte aligned");
        const size_t RR = (size_t)sol->R * sol->R;
        sol->h.pairkey = (unsigned long long *)ws;
        sol->h.msel = (int32_t *)((char *)ws + align_up(RR * 8, 256));
        sol->h.gen = 1;
        k_fill_u64<<<(int)std::min<size_t>((RR + 255) / 256, 1024), 256, 0, st>>>(sol->h.pairkey, RR);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(sol->d, &sol->h, sizeof(SolDev), hipMemcpyHostToDevice, st));
    k_pen_init<<<1, kApplyThreads, 0, st>>>(sol->d);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return TGA_OK;
}

extern "C" int tga_solution_select_moves(tga_solution_t sol, tga_move_t *moves, int32_t cap, int32_t *count,
                                         void *stream) {
    if (!sol || !count || (cap > 0 && !moves) || cap < 0) return fail(TGA_EINVAL, "bad argument");
    if (!sol->h.pairkey) return fail(TGA_EINVAL, "tga_solution_set_multi first");
    hipStream_t st = (hipStream_t)stream;
    k_multi_step<<<1, kApplyThreads, 0, st>>>(sol->d, kModeRecord, TGA_OP_ALL);
    HIPCHK(hipGetLastError());
    std::vector<int32_t> sel(1 + 2 * (size_t)sol->R);
    HIPCHK(hipMemcpyAsync(sel.data(), sol->h.msel, sel.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int ns = sel[0];
    *count = ns;
    const uint32_t Q = (uint32_t)sol->Q;
    for (int q = 0; q < std::min(ns, cap); ++q) {
        const uint32_t id = (uint32_t)sel[1 + 2 * q];
        tga_move_t &m = moves[q];
        m.op = (int32_t)(id / (Q * Q) / 4);
        m.k = (int32_t)(id / (Q * Q) % 4);
        m.a = (int32_t)(id % (Q * Q) / Q);
        m.b = (int32_t)(id % Q);
        m.delta = sel[2 + 2 * q];
        m.feas = 3;
        m.id = id;
        m.version = sol->version;
    }
    return TGA_OK;
}

extern "C" int tga_solution_multi_stats(tga_solution_t sol, int64_t out[2], void *stream) {
    if (!sol || !out) return fail(TGA_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    int32_t steps = 0;
    long long applied = 0;
    HIPCHK(hipMemcpyAsync(&steps, sol->h.state + kStSteps, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&applied, sol->h.acc + kAccMultiApplied, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out[0] = steps;
    out[1] = applied;
    return TGA_OK;
}

// ------------------------------------------------- no-allocation variant ----

// Per-device scratch of tga_eval_routes_static: the solution workspace
// (descriptor, slot attributes, work lists) of the call.  Each GPU the
// library runs on holds one copy until the process ends.  In host code the
// name stands for the host-side shadow, not a device address: kernels and
// copies take the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[TGA_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_ptr(void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TGA_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) return fail(TGA_EDEVICE, "scratch symbol address %p", p);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TGA_OK;
}
}  // namespace

extern "C" int tga_eval_routes_static(tga_instance_t inst, int32_t R, const int32_t *offsets,
                                      const int32_t *customers, uint32_t op_mask, tga_move_t *best,
                                      void *stream) {
    if (!best) return fail(TGA_EINVAL, "null argument");
    if (op_mask & ~TGA_OP_ALL) return fail(TGA_EINVAL, "unknown operator bits 0x%x", op_mask);
    int rc = check_solution_args(inst, R, offsets, customers);
    if (rc) return rc;
    const size_t need = sol_layout(inst->n, R).total;
    if (need > (size_t)TGA_STATIC_SCRATCH_BYTES)
        return fail(TGA_ERANGE, "n = %d, R = %d needs %zu bytes of scratch (maximum %zu)", inst->n, R, need,
                    (size_t)TGA_STATIC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((rc = scratch_ptr(&ws))) return rc;
    hipStream_t st = (hipStream_t)stream;
    tga_solution S{};  // lives for this call only; its arrays are in the scratch
    if ((rc = solution_init(&S, inst, R, offsets, customers, ws, st))) return rc;
    int32_t host[12];  // record and state[0..3]: pageable, so nothing is allocated
    return eval_record(&S, op_mask, best, nullptr, nullptr, st, host, false);
}

extern "C" int tga_apply_move(tga_solution_t sol, const tga_move_t *move, int64_t *new_cost, void *stream) {
    if (!sol || !move) return fail(TGA_EINVAL, "null argument");
    if (sol->in_batch) return fail(TGA_EINVAL, "solution belongs to a batch");
    if (move->version != sol->version)
        return fail(TGA_ESTALE, "move version %u != solution version %u", move->version, sol->version);
    const uint64_t qq = (uint64_t)sol->Q * sol->Q;
    if ((uint64_t)move->id >= 40 * qq) return fail(TGA_EINVAL, "move id %u out of range", move->id);
    hipStream_t st = (hipStream_t)stream;
    void *pin;
    int rc = pinned(&pin);
    if (rc) return rc;
    int32_t *p = (int32_t *)pin;
    p[0] = move->op;
    p[1] = move->k;
    p[2] = move->a;
    p[3] = move->b;
    p[4] = move->delta;
    p[5] = (int32_t)move->feas;
    p[6] = (int32_t)move->id;
    p[7] = (int32_t)move->version;
    HIPCHK(hipMemcpyAsync(sol->h.rec, p, 32, hipMemcpyHostToDevice, st));
    k_finalize<<<1, kApplyThreads, 0, st>>>(sol->d, kModeApplyRec, TGA_OP_ALL, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(p + 8, sol->h.state, 4 * 16 + 8, hipMemcpyDeviceToHost, st));  // state, acc[0]
    HIPCHK(hipStreamSynchronize(st));
    if (p[8 + kStStatus] != 0) return fail(TGA_EINVAL, "move id %u is not a move of N(S)", move->id);
    sol->version++;
    if (new_cost) *new_cost = *(long long *)(p + 8 + 16);
    return TGA_OK;
}

extern "C" int tga_ls_run(tga_solution_t sol, uint32_t op_mask, int32_t max_steps, int32_t *steps_done,
                          int64_t *moves_evaluated, int64_t *cost, void *stream) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    if (sol->in_batch) return fail(TGA_EINVAL, "solution belongs to a batch");
    int rc = check_mask(sol, op_mask);
    if (rc) return rc;
    if (max_steps < 0) return fail(TGA_EINVAL, "max_steps < 0");
    hipStream_t st = (hipStream_t)stream;
    void *pin;
    if ((rc = pinned(&pin))) return rc;
    int32_t *p = (int32_t *)pin;
    k_reset_state<<<1, 64, 0, st>>>(sol->d, 1, max_steps);
    HIPCHK(hipGetLastError());
    const bool multi = (op_mask & TGA_OP_MULTI) != 0;
    if (multi) {  // the per-route-pair table starts empty
        const size_t RR = (size_t)sol->R * sol->R;
        k_fill_u64<<<(int)std::min<size_t>((RR + 255) / 256, 1024), 256, 0, st>>>(sol->h.pairkey, RR);
        HIPCHK(hipGetLastError());
    }
    const int chunk = 16;
    int launched = 0;
    // max_steps evaluations suffice: an evaluation either finds no improving
    // move (converged) or leads to an accepted move, and the cap marks the
    // solution converged after the max_steps-th accepted move
    while (launched < max_steps) {
        const int todo = std::min(chunk, max_steps - launched);
        for (int i = 0; i < todo; ++i) {
            launch_solution_eval(sol, op_mask | kImprovingOnly, nullptr, nullptr, st);
            if (multi)
                k_multi_step<<<1, kApplyThreads, 0, st>>>(sol->d, kModeLS, op_mask);
            else
                k_finalize<<<1, kApplyThreads, 0, st>>>(sol->d, kModeLS, op_mask, nullptr);
        }
        HIPCHK(hipGetLastError());
        launched += todo;
        HIPCHK(hipMemcpyAsync(p, sol->h.state, 64, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (p[kStDone]) break;
    }
    HIPCHK(hipMemcpyAsync(p, sol->h.state, 64 + 8 * kAccCount, hipMemcpyDeviceToHost, st));  // state, acc
    HIPCHK(hipStreamSynchronize(st));
    const long long *acc = (const long long *)(p + 16);
    sol->version = (uint32_t)p[kStVersion];
    if (steps_done) *steps_done = p[kStSteps];
    if (moves_evaluated) *moves_evaluated = acc[kAccMoves];
    if (cost) *cost = acc[kAccCost];
    return TGA_OK;
}

extern "C" int tga_get_solution(tga_solution_t sol, int32_t *offsets, int32_t *customers, int64_t *cost,
                                void *stream) {
    if (!sol || !offsets || !customers) return fail(TGA_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    const int Q = sol->Q, R = sol->R;
    std::vector<int4> a4(Q);
    std::vector<int32_t> roff(R + 1);
    long long c = 0;
    HIPCHK(hipMemcpyAsync(a4.data(), sol->h.a4, sizeof(int4) * Q, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(roff.data(), sol->h.roff, sizeof(int32_t) * (R + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&c, sol->h.acc + kAccCost, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int w = 0;
    for (int r = 0; r < R; ++r) {
        offsets[r] = w;
        for (int s = roff[r] + 1; s < roff[r + 1]; ++s) customers[w++] = a4[s].x & 0xFFFF;
    }
    offsets[R] = w;
    if (cost) *cost = c;
    return TGA_OK;
}

extern "C" int tga_solution_stats(tga_solution_t sol, int32_t *steps_done, int32_t *converged,
                                  int64_t *moves_evaluated, int64_t *cost, void *stream) {
    if (!sol) return fail(TGA_EINVAL, "null solution");
    hipStream_t st = (hipStream_t)stream;
    void *pin;
    int rc = pinned(&pin);
    if (rc) return rc;
    int32_t *p = (int32_t *)pin;
    HIPCHK(hipMemcpyAsync(p, sol->h.state, 64 + 8 * kAccCount, hipMemcpyDeviceToHost, st));  // state, acc
    HIPCHK(hipStreamSynchronize(st));
    const long long *acc = (const long long *)(p + 16);
    sol->version = (uint32_t)p[kStVersion];
    if (steps_done) *steps_done = p[kStSteps];
    if (converged) *converged = p[kStDone];
    if (moves_evaluated) *moves_evaluated = acc[kAccMoves];
    if (cost) *cost = acc[kAccCost];
    return TGA_OK;
}

extern "C" int tga_solution_screen_stats(tga_solution_t sol, int64_t pairs[2], void *stream) {
    if (!sol || !pairs) return fail(TGA_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    long long v[2];
    HIPCHK(hipMemcpyAsync(v, sol->h.acc + kAccFullPairs, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    pairs[0] = v[0];
    pairs[1] = v[1];
    return TGA_OK;
}

extern "C" int tga_move_counts(tga_solution_t sol, int64_t counts[5], void *stream) {
    if (!sol || !counts) return fail(TGA_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    long long acc[kAccCount];
    HIPCHK(hipMemcpyAsync(acc, sol->h.acc, sizeof acc, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < 5; ++i) counts[i] = acc[kAccCnt0 + i];
    return TGA_OK;
}

// ---------------------------------------------------------------- batch ----

struct BatchLayout {
    size_t desc, items, intra, sched, coll, total;
};

// Workspace of a batch of `count` solution slots with room for `max_items`
// inter-route items and `nintra` intra-route groups.
static BatchLayout batch_layout(size_t count, int max_items, int nintra) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.desc = take(sizeof(SolDev) * count);
    L.items = take(sizeof(InterItem) * std::max(max_items, 1));
    L.intra = take(sizeof(IntraItem) * std::max(nintra, 1));
    // item list offsets, done flags, step counter, item queue counters
    L.sched = take(4 * (kMaxBatchGrid + 1) + 4 * (kMaxXcds + 1) + 4 * (count + 1) + 8 * kMaxXcds);
    L.coll = take(32 * count);  // collected results
    L.total = off;
    return L;
}

// Workgroups of kInterThreads threads one compute unit holds at once for
// kernel f with `lds` bytes of dynamic LDS (at least 1).
static int resident_blocks(const void *f, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kInterThreads, lds) != hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    return std::max(1, nb);
}

static int batch_max_items(const std::vector<tga_solution *> &sols, int rows_per_item) {
    long long m = 0;
    for (auto *s : sols)
        if (s) m += count_items(s->Q, rows_per_item > 0 ? rows_per_item : 1);
    return (int)std::min<long long>(m, 1 << 30);
}

extern "C" size_t tga_batch_workspace_bytes(const tga_solution_t *sols, int32_t count) {
    if (!sols || count < 1) return 0;
    std::vector<tga_solution *> v(sols, sols + count);
    int nintra = 0;
    for (auto *s : v) {
        if (!s) return 0;
        nintra += s->R;
    }
    // worst case over the schedules tga_batch_create accepts: one row per item
    return batch_layout(v.size(), batch_max_items(v, 1), nintra).total;
}

// Rows per inter-route item of the batched form when none are given: one
// LDS sub-block, or for large solutions (fewer than kItemRowsMin rows per
// sub-block) several whole sub-blocks, so that the two boundary rows carried
// from one sub-block to the next spare re-reading them (a one-row sub-block
// would otherwise read every row three times).  No more than that: a single
// solution of 10^4 customers on the whole LDS (6-row sub-blocks) evaluates
// in 147 us with 12-row items against 162 us with 18-row ones, which leave
// its 256 workgroups about two items each.
constexpr int kItemRowsMin = 12;
static int default_item_rows(int tile_rows, int tuned) {
    if (tuned > 0)  // tuned: thin items within one sub-block, else whole sub-blocks
        return tuned <= tile_rows ? tuned : tile_rows * ((tuned + tile_rows - 1) / tile_rows);
    if (tile_rows >= kItemRowsMin) return tile_rows;
    return tile_rows * ((kItemRowsMin + tile_rows - 1) / tile_rows);
}

// Rows per LDS sub-block for an LDS budget of `budget` bytes.
static int tile_rows_for(int np1, bool w16, size_t budget) {
    int h = 1;
    while (h < kMaxTileRows && rows_lds(np1, h + 1, w16) <= budget) ++h;
    return h;
}

static void drop_tick_graph(tga_batch *B) {
    if (B->tick_exec) (void)hipGraphExecDestroy(B->tick_exec);
    if (B->tick_graph) (void)hipGraphDestroy(B->tick_graph);
    B->tick_exec = nullptr;
    B->tick_graph = nullptr;
    B->tick_steps = -1;
}

// Upload a slot batch's plan without synchronising the host: the plan is
// written into one of two pinned staging buffers (taken in turn; the host
// waits only if that buffer's previous upload has not run yet) and copied on
// `st`, so it takes effect for the launches enqueued after it.
static int stage_upload(tga_batch *B, const std::vector<SolDev> &descs, const std::vector<InterItem> &items,
                        const std::vector<IntraItem> &intra, const std::vector<int> &woff,
                        const std::vector<int> &ixoff, hipStream_t st) {
    const size_t nd = sizeof(SolDev) * descs.size(), ni = sizeof(InterItem) * items.size(),
                 ng = sizeof(IntraItem) * intra.size(), nw = sizeof(int) * woff.size(),
                 nx = sizeof(int) * ixoff.size();
    const size_t od = 0, oi = align_up(od + nd, 64), og = align_up(oi + ni, 64), ow = align_up(og + ng, 64),
                 ox = align_up(ow + nw, 64), total = ox + nx;
    if (total > B->stage_bytes) return fail(TGA_ERANGE, "plan of %zu bytes exceeds the staging buffer", total);
    const int k = B->stage_k;
    B->stage_k ^= 1;
    HIPCHK(hipEventSynchronize(B->stage_ev[k]));
    char *h = B->stage_h[k];
    memcpy(h + od, descs.data(), nd);
    if (ni) memcpy(h + oi, items.data(), ni);
    if (ng) memcpy(h + og, intra.data(), ng);
    memcpy(h + ow, woff.data(), nw);
    memcpy(h + ox, ixoff.data(), nx);
    HIPCHK(hipMemcpyAsync(B->d, h + od, nd, hipMemcpyHostToDevice, st));
    if (ni) HIPCHK(hipMemcpyAsync(B->items, h + oi, ni, hipMemcpyHostToDevice, st));
    if (ng) HIPCHK(hipMemcpyAsync(B->intra, h + og, ng, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(B->woff, h + ow, nw, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(B->ixoff, h + ox, nx, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(B->stage_ev[k], st));
    return TGA_OK;
}

// Plan the batch's schedule for its configuration and upload it: the
// descriptors (with their rows per sub-block) and the per-XCD item lists.
// The workspace regions hold the worst case of every configuration.
static int batch_plan(tga_batch *B, const DevProps &P, hipStream_t st) {
    const std::vector<tga_solution *> &v = B->sols;
    const int count = (int)v.size();
    const tga_batch_config_t &c = B->cfg;
    std::vector<InterItem> items;
    std::vector<IntraItem> intra;
    std::vector<SolDev> descs(count);
    size_t lds = 0;
    std::vector<int> trs(count, 0);
    for (int i = 0; i < count; ++i) {
        tga_solution *s = v[i];
        if (!s) {  // empty slot: Q = 0, no items; the per-solution kernels skip it
            memset(&descs[i], 0, sizeof(SolDev));
            continue;
        }
        descs[i] = s->h;
        // LDS sub-block rows (bounded by the LDS budget of one workgroup)
        const bool w16 = s->h.D16 != nullptr;
        const int cap_rows = tile_rows_for(s->h.np1, w16, (size_t)c.lds_kb * 1024);
        const int tr = c.sub_rows > 0 ? std::min(c.sub_rows, cap_rows) : cap_rows;
        trs[i] = tr;
        descs[i].tile_rows = tr;
        lds = std::max(lds, rows_lds(s->h.np1, tr, w16));
    }
    const size_t lds_intra = (size_t)kInterWaves * kIntraRegionBytes;  // the intra phase's regions
    if (!c.split) lds = std::max(lds, lds_intra);
    // A slot batch keeps its launch shapes while members come and go (so a
    // captured tick stays valid): LDS at least the configured budget, and
    // never below what earlier members needed.
    if (B->slotted) lds = std::max(lds, std::max((size_t)c.lds_kb * 1024, B->lds));
    if (lds > (size_t)P.max_lds) return fail(TGA_ERANGE, "batch needs %zu bytes of LDS", lds);
    // one resident wave of workgroups: as many as LDS and registers allow
    const int grid_inter =
        P.cus * resident_blocks(c.split ? (const void *)k_eval_batch<1> : (const void *)k_eval_batch<3>, lds);
    const int grid_intra = P.cus * resident_blocks((const void *)k_eval_batch<2>, lds_intra);
    // Workgroups of a resident grid are dispatched round-robin over the XCDs
    // (each with its own L2), so workgroup b works on the item list of XCD
    // b mod nx.  A solution is placed on one XCD (largest first, onto the
    // least loaded one), so that its attributes and halo rows stay in one L2,
    // unless it holds more than half of an XCD's fair share of the work: then
    // its strips are split into contiguous ranges of about a quarter of that
    // share, each placed the same way, and its intra-route groups are dealt
    // round-robin (one large request must not be confined to one XCD).
    // Inter-route items are strips of rows of one solution (one LDS sub-block
    // each by default); each list is sorted largest first (rows times the
    // columns to their right), ties in solution / row order.
    const int nx = (grid_inter % kMaxXcds == 0 && grid_intra % kMaxXcds == 0) ? kMaxXcds : 1;
    auto work = [&](const InterItem &a) {
        const long long Q = v[a.sol]->Q, r = a.s1 - a.s0;
        return r * (2 * Q - a.s0 - a.s1 + 1);
    };
    // a VRPTW pair costs more than a CVRP one (window tests, more routes and
    // their walks): the XCD placement weighs VRPTW work 1.1, which evens the
    // XCDs' finishing times on mixed batches
    auto tw_weight = [&](int i) { return v[i]->h.has_tw ? 1.1 : 1.0; };
    std::vector<std::vector<InterItem>> own(count);
    std::vector<double> sol_work(count, 0.0);
    double total = 0.0;
    for (int i = 0; i < count; ++i) {
        if (!v[i]) continue;
        for_each_item(v[i]->Q, c.rows_per_item > 0 ? c.rows_per_item : default_item_rows(trs[i], v[i]->item_rows),
                      [&](int s0, int s1) { own[i].push_back(InterItem{i, s0, s1, 0}); });
        for (const auto &it : own[i]) sol_work[i] += (double)work(it) * tw_weight(i);
        total += sol_work[i];
    }
    const double share = total / nx;
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sol_work[a] > sol_work[b]; });
    std::vector<double> load(nx, 0.0);
    std::vector<std::vector<InterItem>> xitems(nx);
    std::vector<std::vector<IntraItem>> xintra(nx);
    auto least = [&]() { return (int)(std::min_element(load.begin(), load.end()) - load.begin()); };
    int rr = 0;
    for (int i : order) {
        if (!v[i]) continue;
        std::vector<IntraItem> groups;
        push_intra_groups(v[i]->n, v[i]->R, i, groups);
        if (nx == 1 || sol_work[i] <= 0.5 * share) {
            const int x = least();
            load[x] += sol_work[i];
            xitems[x].insert(xitems[x].end(), own[i].begin(), own[i].end());
            xintra[x].insert(xintra[x].end(), groups.begin(), groups.end());
            continue;
        }
        const double piece = 0.25 * share;
        size_t k = 0;
        while (k < own[i].size()) {
            const int x = least();
            double w = 0.0;
            do {
                w += (double)work(own[i][k]) * tw_weight(i);
                xitems[x].push_back(own[i][k++]);
            } while (k < own[i].size() && w < piece);
            load[x] += w;
        }
        for (const auto &g : groups) xintra[rr++ % nx].push_back(g);
    }
    // Within an XCD, the workgroups take the items from one queue, largest
    // first (the evaluation launch pulls them with an atomic counter), so the
    // work of a step spreads over the XCD's workgroups whatever the items
    // and the intra-route groups cost and whichever solutions have converged.
    if (grid_inter > kMaxBatchGrid) return fail(TGA_ERANGE, "batch grid of %d workgroups", grid_inter);
    std::vector<int> woff(nx + 1, 0), ixoff(nx + 1, 0);
    for (int x = 0; x < nx; ++x) {
        std::stable_sort(xitems[x].begin(), xitems[x].end(),
                         [&](const InterItem &a, const InterItem &b) { return work(a) > work(b); });
        items.insert(items.end(), xitems[x].begin(), xitems[x].end());
        woff[x + 1] = (int)items.size();
        intra.insert(intra.end(), xintra[x].begin(), xintra[x].end());
        ixoff[x + 1] = (int)intra.size();
    }
    if ((int)items.size() > B->max_items || (int)intra.size() > B->max_intra)
        return fail(TGA_ERANGE, "batch schedule exceeds its workspace");
    const bool shapes_same = B->nx == nx && B->lds == lds && B->lds_intra == lds_intra &&
                             B->grid_inter == grid_inter && B->grid_intra == grid_intra;
    B->nitems = (int)items.size();
    B->nintra = (int)intra.size();
    B->nx = nx;
    B->lds = lds;
    B->lds_intra = lds_intra;
    B->grid_inter = grid_inter;
    B->grid_intra = grid_intra;
    // A captured step loop holds the old launch shapes and the old
    // membership; a captured tick of a slot batch reads the membership from
    // the workspace and stays valid while the shapes do.
    if (B->exec) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    if (B->graph) {
        (void)hipGraphDestroy(B->graph);
        B->graph = nullptr;
    }
    B->graph_steps = -1;
    if (!shapes_same) drop_tick_graph(B);
    if (B->slotted) return stage_upload(B, descs, items, intra, woff, ixoff, st);
    hipError_t e = hipMemcpyAsync(B->d, descs.data(), sizeof(SolDev) * count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->items, items.data(), sizeof(InterItem) * items.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !intra.empty())
        e = hipMemcpyAsync(B->intra, intra.data(), sizeof(IntraItem) * intra.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->woff, woff.data(), sizeof(int) * woff.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(B->steps, 0, sizeof(int32_t), st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->ixoff, ixoff.data(), sizeof(int) * (nx + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(TGA_EDEVICE, "batch plan: %s", hipGetErrorString(e));
    return TGA_OK;
}

static int check_config(const tga_batch_config_t &c) {
    if (c.rows_per_item < 0 || c.rows_per_item > 256 || c.sub_rows < 0 || c.sub_rows > 64)
        return fail(TGA_ERANGE, "rows_per_item in [0, 256], sub_rows in [0, 64]");
    if (c.lds_kb < 8 || c.lds_kb > 160) return fail(TGA_ERANGE, "lds_kb in [8, 160]");
    if (c.split != 0 && c.split != 1) return fail(TGA_EINVAL, "split must be 0 or 1");
    return TGA_OK;
}

// Release what a batch owns on the host side (pinned buffers, events,
// graphs, the capture stream) and the batch itself.
static void batch_destroy(tga_batch *B) {
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    drop_tick_graph(B);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    if (B->coll_h) (void)hipHostFree(B->coll_h);
    for (int k = 0; k < 2; ++k) {
        if (B->stage_ev[k]) (void)hipEventDestroy(B->stage_ev[k]);
        if (B->tick_ev[k]) (void)hipEventDestroy(B->tick_ev[k]);
        if (B->stage_h[k]) (void)hipHostFree(B->stage_h[k]);
        if (B->tick_h[k]) (void)hipHostFree(B->tick_h[k]);
    }
    for (auto *s : B->sols)
        if (s) s->in_batch = 0;
    delete B;
}

// Common set-up of both kinds of batch: workspace layout for `count` slots,
// the pinned result buffer, and (slot batches) the staging buffers and
// events; then the first plan.
static int batch_init(tga_batch *B, int max_items, int nintra, void *ws, hipStream_t st) {
    const size_t count = B->sols.size();
    const BatchLayout L = batch_layout(count, max_items, nintra);
    char *base = (char *)ws;
    B->d = (SolDev *)(base + L.desc);
    B->items = (InterItem *)(base + L.items);
    B->max_items = max_items;
    B->intra = (IntraItem *)(base + L.intra);
    B->max_intra = nintra;
    B->woff = (int *)(base + L.sched);
    B->ixoff = B->woff + (kMaxBatchGrid + 1);
    B->done = B->ixoff + (kMaxXcds + 1);
    B->steps = B->done + count;
    B->qctr = (uint32_t *)(B->steps + 1);
    B->coll = (long long *)(base + L.coll);
    B->exec = nullptr;
    B->graph = nullptr;
    B->graph_steps = -1;
    B->cap_stream = nullptr;
    if (hipHostMalloc((void **)&B->coll_h, 32 * count, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        B->coll_h = nullptr;
        return fail(TGA_ENOMEM, "pinned host buffer of %zu bytes", 32 * count);
    }
    if (B->slotted) {
        B->stage_bytes = sizeof(SolDev) * count + sizeof(InterItem) * max_items + sizeof(IntraItem) * nintra +
                         4 * (kMaxBatchGrid + 1) + 4 * (kMaxXcds + 1) + 5 * 64;
        for (int k = 0; k < 2; ++k) {
            if (hipHostMalloc((void **)&B->stage_h[k], B->stage_bytes, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void **)&B->tick_h[k], 32 * count, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return fail(TGA_ENOMEM, "pinned staging buffers");
            }
            HIPCHK(hipEventCreateWithFlags(&B->stage_ev[k], hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&B->tick_ev[k], hipEventDisableTiming));
        }
        k_zero_i32<<<1, 64, 0, st>>>(B->steps, 1);
        HIPCHK(hipGetLastError());
    }
    k_zero_i32<<<1, 64, 0, st>>>((int32_t *)B->qctr, 2 * kMaxXcds);  // then kept at zero by the launches
    HIPCHK(hipGetLastError());
    DevProps P;
    int rc = props(&P);
    if (rc) return rc;
    return batch_plan(B, P, st);
}

static tga_batch_config_t default_config(int32_t rows_per_item, int32_t sub_rows) {
    tga_batch_config_t cfg;
    cfg.lds_kb = (int32_t)(lds_budget() / 1024);
    cfg.split = 0;
    cfg.rows_per_item = rows_per_item;
    cfg.sub_rows = sub_rows;
    cfg.us_per_eval = 0.f;
    return cfg;
}

extern "C" int tga_batch_create(const tga_solution_t *sols, int32_t count, int32_t rows_per_item,
                                int32_t sub_rows, void *ws, size_t ws_bytes, void *stream,
                                tga_batch_t *out) {
    if (!out) return fail(TGA_EINVAL, "out is null");
    *out = nullptr;
    if (!sols || count < 1 || !ws) return fail(TGA_EINVAL, "bad batch arguments");
    const tga_batch_config_t cfg = default_config(rows_per_item, sub_rows);
    int rc = check_config(cfg);
    if (rc) return rc;
    if (((uintptr_t)ws) & 255) return fail(TGA_EINVAL, "workspace must be 256-byte aligned");
    std::vector<tga_solution *> v(sols, sols + count);
    for (auto *s : v) {
        if (!s) return fail(TGA_EINVAL, "null solution in batch");
        if (s->in_batch) return fail(TGA_EINVAL, "solution already in a batch");
        if (s->h.pen || s->h.pd || s->h.gen)
            return fail(TGA_EINVAL, "solutions on the general path are evaluated one at a time");
    }
    for (size_t i = 0; i < v.size(); ++i)
        for (size_t j = i + 1; j < v.size(); ++j)
            if (v[i] == v[j]) return fail(TGA_EINVAL, "solution listed twice");
    if (ws_bytes < tga_batch_workspace_bytes(sols, count)) return fail(TGA_ENOMEM, "batch workspace too small");
    int nintra = 0;
    for (auto *s : v) nintra += s->R;
    tga_batch *B = new tga_batch();
    B->sols = v;
    B->cfg = cfg;
    if ((rc = batch_init(B, batch_max_items(v, 1), nintra, ws, (hipStream_t)stream))) {
        B->sols.assign(v.size(), nullptr);  // not members yet
        batch_destroy(B);
        return rc;
    }
    for (auto *s : v) s->in_batch = 1;
    *out = B;
    return TGA_OK;
}

extern "C" size_t tga_batch_slots_workspace_bytes(int32_t slots, int32_t max_sum_q, int32_t max_sum_r) {
    if (slots < 1 || slots > kMaxSlots || max_sum_q < 1 || max_sum_r < 1) return 0;
    return batch_layout((size_t)slots, max_sum_q, max_sum_r).total;
}

extern "C" int tga_batch_create_slots(int32_t slots, int32_t max_sum_q, int32_t max_sum_r, void *ws,
                                      size_t ws_bytes, void *stream, tga_batch_t *out) {
    if (!out) return fail(TGA_EINVAL, "out is null");
    *out = nullptr;
    if (!ws) return fail(TGA_EINVAL, "null workspace");
    if (slots < 1 || slots > kMaxSlots) return fail(TGA_ERANGE, "slots = %d outside [1, %d]", slots, kMaxSlots);
    if (max_sum_q < 1 || max_sum_r < 1) return fail(TGA_ERANGE, "max_sum_q and max_sum_r must be positive");
    if (((uintptr_t)ws) & 255) return fail(TGA_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < tga_batch_slots_workspace_bytes(slots, max_sum_q, max_sum_r))
        return fail(TGA_ENOMEM, "batch workspace too small");
    tga_batch *B = new tga_batch();
    B->sols.assign(slots, nullptr);
    B->cfg = default_config(0, 0);
    B->slotted = 1;
    B->max_sum_q = max_sum_q;
    B->max_sum_r = max_sum_r;
    int rc = batch_init(B, max_sum_q, max_sum_r, ws, (hipStream_t)stream);
    if (rc) {
        batch_destroy(B);
        return rc;
    }
    *out = B;
    return TGA_OK;
}

extern "C" int tga_batch_set_members(tga_batch_t B, const tga_solution_t *sols, void *stream) {
    if (!B || !sols) return fail(TGA_EINVAL, "null argument");
    if (!B->slotted) return fail(TGA_EINVAL, "not a slot batch");
    const int slots = (int)B->sols.size();
    long long sq = 0, sr = 0;
    for (int i = 0; i < slots; ++i) {
        tga_solution *s = sols[i];
        if (!s) continue;
        bool ours = false;
        for (auto *o : B->sols) ours = ours || o == s;
        if (s->in_batch && !ours) return fail(TGA_EINVAL, "solution in slot %d belongs to another batch", i);
        if (s->h.pen || s->h.pd || s->h.gen)
            return fail(TGA_EINVAL, "solutions on the general path are evaluated one at a time");
        for (int j = 0; j < i; ++j)
            if (sols[j] == s) return fail(TGA_EINVAL, "solution listed in slots %d and %d", j, i);
        sq += s->Q;
        sr += s->R;
    }
    if (sq > B->max_sum_q || sr > B->max_sum_r)
        return fail(TGA_ERANGE, "members hold Q = %lld, R = %lld (room for %d, %d)", sq, sr, B->max_sum_q,
                    B->max_sum_r);
    std::vector<tga_solution *> old = B->sols;
    for (auto *o : old)
        if (o) o->in_batch = 0;
    B->sols.assign(sols, sols + slots);
    DevProps P;
    int rc = props(&P);
    if (!rc) rc = batch_plan(B, P, (hipStream_t)stream);
    if (rc) {
        B->sols = old;
        for (auto *o : old)
            if (o) o->in_batch = 1;
        return rc;
    }
    for (auto *s : B->sols)
        if (s) s->in_batch = 1;
    return TGA_OK;
}

// `ls`: the evaluation feeds a local-search step (only an improving move can
// be applied), see kImprovingOnly.
static void batch_eval_launch(tga_batch *B, uint32_t op_mask, bool ls, hipStream_t st) {
    if (!(op_mask & TGA_OP_ALL)) return;
    if (ls) op_mask |= kImprovingOnly;
    const bool cnt = ls && (op_mask & TGA_OP_COUNT_FULL);
    if (!B->cfg.split) {
        if (cnt)
            k_eval_batch<7><<<B->grid_inter, kInterThreads, B->lds, st>>>(B->d, B->items, B->woff, B->qctr,
                                                                         B->intra, B->ixoff, B->nx, op_mask);
        else
            k_eval_batch<3><<<B->grid_inter, kInterThreads, B->lds, st>>>(B->d, B->items, B->woff, B->qctr,
                                                                         B->intra, B->ixoff, B->nx, op_mask);
        return;
    }
    if ((op_mask & 7) && cnt)
        k_eval_batch<5><<<B->grid_inter, kInterThreads, B->lds, st>>>(B->d, B->items, B->woff, B->qctr,
                                                                     B->intra, B->ixoff, B->nx, op_mask);
    else if (op_mask & 7)
        k_eval_batch<1><<<B->grid_inter, kInterThreads, B->lds, st>>>(B->d, B->items, B->woff, B->qctr,
                                                                     B->intra, B->ixoff, B->nx, op_mask);
    if (op_mask & (2 | 8 | 16))
        k_eval_batch<2><<<B->grid_intra, kInterThreads, B->lds_intra, st>>>(
            B->d, B->items, B->woff, B->qctr, B->intra, B->ixoff, B->nx, op_mask);
}

static void batch_finalize_launch(tga_batch *B, uint32_t op_mask, int mode, hipStream_t st) {
    k_finalize<<<(int)B->sols.size(), kApplyThreads, 0, st>>>(B->d, mode, op_mask, B->steps);
}

static void batch_step(tga_batch *B, uint32_t op_mask, int mode, hipStream_t st) {
    batch_eval_launch(B, op_mask, mode == kModeLS, st);
    batch_finalize_launch(B, op_mask, mode, st);
}

extern "C" int tga_batch_get_config(tga_batch_t B, tga_batch_config_t *out) {
    if (!B || !out) return fail(TGA_EINVAL, "null argument");
    *out = B->cfg;
    return TGA_OK;
}

extern "C" int tga_batch_set_config(tga_batch_t B, const tga_batch_config_t *cfg, void *stream) {
    if (!B || !cfg) return fail(TGA_EINVAL, "null argument");
    int rc = check_config(*cfg);
    if (rc) return rc;
    DevProps P;
    if ((rc = props(&P))) return rc;
    const tga_batch_config_t old = B->cfg;
    B->cfg = *cfg;
    B->cfg.us_per_eval = 0.f;
    B->lds = 0;  // a new schedule sets the LDS of a slot batch afresh
    if ((rc = batch_plan(B, P, (hipStream_t)stream))) {
        B->cfg = old;  // keep (and re-upload) the previous schedule
        const std::string msg = tga_last_error();
        if (batch_plan(B, P, (hipStream_t)stream) != TGA_OK) return rc;
        return fail(rc, "%s", msg.c_str());
    }
    return TGA_OK;
}

extern "C" int tga_batch_autotune(tga_batch_t B, uint32_t op_mask, int32_t launches, tga_batch_config_t *best,
                                  void *stream) {
    if (!B) return fail(TGA_EINVAL, "null batch");
    if (op_mask & ~TGA_OP_ALL) return fail(TGA_EINVAL, "unknown operator bits 0x%x", op_mask);
    if (launches < 1 || launches > 1000) return fail(TGA_ERANGE, "launches in [1, 1000]");
    DevProps P;
    int rc = props(&P);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(TGA_EDEVICE, "hipEventCreate failed");
    }
    const tga_batch_config_t base = B->cfg;
    // LDS budgets per inter-route workgroup: up to the largest that lets two
    // workgroups share a compute unit, and the whole LDS of one workgroup
    // (one per compute unit: fewer, longer-row sub-blocks, which suit very
    // large solutions)
    const int kLdsKb[] = {40, 52, 64, 78, 79, (int)(P.max_lds / 1024)};
    tga_batch_config_t chosen = base;
    float best_us = 0.f;
    bool any = false;
    hipError_t e = hipSuccess;
    for (int split = 0; split <= 1 && e == hipSuccess; ++split) {
        for (int kb : kLdsKb) {
            tga_batch_config_t c = base;
            c.lds_kb = kb;
            c.split = split;
            c.us_per_eval = 0.f;
            B->cfg = c;
            B->lds = 0;
            if (batch_plan(B, P, st) != TGA_OK) continue;  // does not fit this device
            // local-search evaluations, each followed by a finalize that only
            // records (and clears) the best move
            auto step = [&]() {
                batch_eval_launch(B, op_mask, true, st);
                batch_finalize_launch(B, op_mask, kModeRecord, st);
            };
            step();  // untimed
            e = hipEventRecord(e0, st);
            for (int i = 0; i < launches && e == hipSuccess; ++i) step();
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            const float us = ms * 1000.f / launches;
            if (!any || us < best_us) {
                any = true;
                best_us = us;
                chosen = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        B->cfg = base;
        B->lds = 0;
        (void)batch_plan(B, P, st);
        return fail(TGA_EDEVICE, "autotune: %s", hipGetErrorString(e));
    }
    if (!any) {
        B->cfg = base;
        B->lds = 0;
        (void)batch_plan(B, P, st);
        return fail(TGA_ERANGE, "no candidate schedule fits the device");
    }
    chosen.us_per_eval = best_us;
    B->cfg = chosen;
    B->lds = 0;
    if ((rc = batch_plan(B, P, st))) return rc;
    if (best) *best = chosen;
    return TGA_OK;
}

extern "C" int tga_batch_reset(tga_batch_t B, void *stream) {
    if (!B) return fail(TGA_EINVAL, "null batch");
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)B->sols.size();
    k_reset_state<<<(n + 63) / 64, 64, 0, st>>>(B->d, n, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return TGA_OK;
}

// One kernel gathers every solution's results, one copy brings them over.
static int batch_collect(tga_batch *B, int32_t *steps_done, int64_t *moves, int64_t *cost, hipStream_t st) {
    const int n = (int)B->sols.size();
    k_collect<<<(n + 255) / 256, 256, 0, st>>>(B->d, n, B->coll);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(B->coll_h, B->coll, 32 * (size_t)n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
        const long long *r = B->coll_h + 4 * i;
        if (B->sols[i]) B->sols[i]->version = (uint32_t)r[1];  // low half; converged flag above
        if (steps_done) steps_done[i] = (int32_t)r[0];
        if (moves) moves[i] = r[2];
        if (cost) cost[i] = r[3];
    }
    return TGA_OK;
}

extern "C" int tga_probe_stream_read(const void *src, size_t bytes, void *stream) {
    if (!src) return fail(TGA_EINVAL, "null argument");
    if (((uintptr_t)src) & 15) return fail(TGA_EINVAL, "src must be 16-byte aligned");
    if (bytes % 1024) return fail(TGA_EINVAL, "bytes must be a multiple of 1024");
    DevProps P;
    int rc = props(&P);
    if (rc) return rc;
    const long long chunks = (long long)(bytes / 1024);
    if (chunks == 0) return TGA_OK;
    const long long want = (chunks + 3) / 4;
    const int grid = (int)std::max(1LL, std::min<long long>(want, 8LL * P.cus));
    hipStream_t st = (hipStream_t)stream;
    k_probe_stream<<<grid, 256, 0, st>>>((const int *)src, chunks);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return TGA_OK;
}

extern "C" int tga_batch_screen_stats(tga_batch_t B, int64_t pairs[2], void *stream) {
    if (!B || !pairs) return fail(TGA_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    k_screen_sum<<<1, 64, 0, st>>>(B->d, (int)B->sols.size(), B->coll);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(B->coll_h, B->coll, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    pairs[0] = B->coll_h[0];
    pairs[1] = B->coll_h[1];
    return TGA_OK;
}

extern "C" int tga_batch_ls_run(tga_batch_t B, uint32_t op_mask, int32_t steps, int32_t use_graph,
                                int32_t *steps_done, int64_t *moves_evaluated, int64_t *cost, void *stream) {
    if (!B) return fail(TGA_EINVAL, "null batch");
    if (op_mask & ~(TGA_OP_ALL | TGA_OP_COUNT_FULL)) return fail(TGA_EINVAL, "unknown operator bits 0x%x", op_mask);
    if (steps < 0) return fail(TGA_EINVAL, "steps < 0");
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)B->sols.size();
    k_reset_state<<<(n + 63) / 64, 64, 0, st>>>(B->d, n, steps);
    HIPCHK(hipGetLastError());
    // `steps` evaluations per solution suffice (see tga_ls_run)
    const int evals = steps;
    if (use_graph) {
        if (!B->cap_stream) HIPCHK(hipStreamCreate(&B->cap_stream));
        if (!B->exec || B->graph_steps != evals || B->graph_mask != op_mask) {
            if (B->exec) {
                (void)hipGraphExecDestroy(B->exec);
                B->exec = nullptr;
            }
            if (B->graph) {
                (void)hipGraphDestroy(B->graph);
                B->graph = nullptr;
            }
            HIPCHK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < evals; ++i) batch_step(B, op_mask, kModeLS, B->cap_stream);
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamEndCapture(B->cap_stream, &g));
            B->graph = g;
            HIPCHK(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
            B->graph_steps = evals;
            B->graph_mask = op_mask;
        }
        HIPCHK(hipGraphLaunch(B->exec, st));
    } else {
        for (int i = 0; i < evals; ++i) batch_step(B, op_mask, kModeLS, st);
        HIPCHK(hipGetLastError());
    }
    return batch_collect(B, steps_done, moves_evaluated, cost, st);
}

extern "C" int tga_batch_begin(tga_batch_t B, int32_t max_steps, void *stream) {
    if (!B) return fail(TGA_EINVAL, "null batch");
    if (max_steps < 0) return fail(TGA_EINVAL, "max_steps < 0");
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)B->sols.size();
    k_reset_state<<<(n + 63) / 64, 64, 0, st>>>(B->d, n, max_steps);
    HIPCHK(hipGetLastError());
    return TGA_OK;
}

extern "C" int tga_batch_poll(tga_batch_t B, int32_t *done, void *stream) {
    if (!B || !done) return fail(TGA_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)B->sols.size();
    k_poll_done<<<(n + 255) / 256, 256, 0, st>>>(B->d, n, B->done);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(done, B->done, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return TGA_OK;
}

extern "C" int tga_batch_step_part(tga_batch_t B, uint32_t op_mask, int32_t part, void *stream) {
    if (!B) return fail(TGA_EINVAL, "null batch");
    if (op_mask & ~(TGA_OP_ALL | TGA_OP_COUNT_FULL)) return fail(TGA_EINVAL, "unknown operator bits 0x%x", op_mask);
    if (part != 0 && part != 1) return fail(TGA_EINVAL, "part must be 0 (evaluate) or 1 (finalize)");
    hipStream_t st = (hipStream_t)stream;
    if (part == 0)
        batch_eval_launch(B, op_mask, true, st);
    else
        batch_finalize_launch(B, op_mask, kModeLS, st);
    HIPCHK(hipGetLastError());
    return TGA_OK;
}

extern "C" int tga_batch_collect(tga_batch_t B, int32_t *steps_done, int64_t *moves_evaluated, int64_t *cost,
                                 void *stream) {
    if (!B) return fail(TGA_EINVAL, "null batch");
    return batch_collect(B, steps_done, moves_evaluated, cost, (hipStream_t)stream);
}

extern "C" int tga_batch_eval(tga_batch_t B, uint32_t op_mask, tga_move_t *best, int32_t *status, void *stream) {
    if (!B || !best) return fail(TGA_EINVAL, "null argument");
    if (op_mask & ~(TGA_OP_ALL | TGA_OP_COUNT_FULL)) return fail(TGA_EINVAL, "unknown operator bits 0x%x", op_mask);
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)B->sols.size();
    // a record evaluation covers converged solutions too, so their flags and
    // counters stay as they are
    batch_step(B, op_mask, kModeRecord, st);
    HIPCHK(hipGetLastError());
    std::vector<int32_t> rec(8 * n, 0), state(16 * n, 0);
    for (int i = 0; i < n; ++i) {
        if (!B->sols[i]) continue;
        HIPCHK(hipMemcpyAsync(&rec[8 * i], B->sols[i]->h.rec, 32, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(&state[16 * i], B->sols[i]->h.state, 64, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
        to_move(&rec[8 * i], &best[i]);
        if (!B->sols[i]) {  // empty slot
            if (status) status[i] = 1;
            continue;
        }
        best[i].version = B->sols[i]->version;
        if (status) status[i] = state[16 * i + kStStatus];
    }
    return TGA_OK;
}

// One tick of a slot batch: `steps` local-search steps of every member (one
// captured graph, replayed), then the per-slot results gathered and copied
// into the pinned buffer of this tick, with an event behind the copy.
extern "C" int tga_batch_tick(tga_batch_t B, uint32_t op_mask, int32_t steps, int32_t *tick, void *stream) {
    if (!B) return fail(TGA_EINVAL, "null batch");
    if (!B->slotted) return fail(TGA_EINVAL, "not a slot batch");
    if (op_mask & ~(TGA_OP_ALL | TGA_OP_COUNT_FULL)) return fail(TGA_EINVAL, "unknown operator bits 0x%x", op_mask);
    if (steps < 1 || steps > 64) return fail(TGA_ERANGE, "steps per tick in [1, 64]");
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)B->sols.size();
    if (!B->tick_exec || B->tick_steps != steps || B->tick_mask != op_mask) {
        drop_tick_graph(B);
        if (!B->cap_stream) HIPCHK(hipStreamCreate(&B->cap_stream));
        HIPCHK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < steps; ++i) batch_step(B, op_mask, kModeLS, B->cap_stream);
        k_collect<<<(n + 255) / 256, 256, 0, B->cap_stream>>>(B->d, n, B->coll);
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamEndCapture(B->cap_stream, &g));
        B->tick_graph = g;
        HIPCHK(hipGraphInstantiate(&B->tick_exec, g, nullptr, nullptr, 0));
        B->tick_steps = steps;
        B->tick_mask = op_mask;
    }
    const int k = B->ticks & 1;
    HIPCHK(hipEventSynchronize(B->tick_ev[k]));  // the buffer's previous tick has been read back
    HIPCHK(hipGraphLaunch(B->tick_exec, st));
    HIPCHK(hipMemcpyAsync(B->tick_h[k], B->coll, 32 * (size_t)n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(B->tick_ev[k], st));
    B->tick_seq[k] = B->ticks;
    if (tick) *tick = B->ticks;
    B->ticks++;
    return TGA_OK;
}

// Results of the newest finished tick, without waiting: *tick = its number
// (-1 when none has finished yet; the arrays are then untouched).
extern "C" int tga_batch_tick_status(tga_batch_t B, int32_t *tick, int32_t *converged, int32_t *steps_done,
                                     int64_t *moves_evaluated, int64_t *cost) {
    if (!B || !tick) return fail(TGA_EINVAL, "null argument");
    if (!B->slotted) return fail(TGA_EINVAL, "not a slot batch");
    *tick = -1;
    const int n = (int)B->sols.size();
    for (int back = 1; back <= 2; ++back) {
        const int t = B->ticks - back;
        if (t < 0) break;
        const int k = t & 1;
        const hipError_t q = hipEventQuery(B->tick_ev[k]);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(TGA_EDEVICE, "tick event: %s", hipGetErrorString(q));
        const long long *r = B->tick_h[k];
        for (int i = 0; i < n; ++i) {
            if (converged) converged[i] = (int32_t)(r[4 * i + 1] >> 32);
            if (steps_done) steps_done[i] = (int32_t)r[4 * i];
            if (moves_evaluated) moves_evaluated[i] = r[4 * i + 2];
            if (cost) cost[i] = r[4 * i + 3];
        }
        *tick = B->tick_seq[k];
        return TGA_OK;
    }
    return TGA_OK;
}

extern "C" int tga_batch_free(tga_batch_t B) {
    if (!B) return TGA_OK;
    batch_destroy(B);
    return TGA_OK;
}
