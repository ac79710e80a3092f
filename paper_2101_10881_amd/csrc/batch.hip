// batch.hip -- many polynomials in one persistent launch.
//
// Every instance keeps its own plan (Section 5 job lists), workspace and
// buffers.  The batch turns all instances' stages -- staging, each
// convolution layer, each addition level, gathering -- into tasks: a task is
// a chunk of one stage of one instance, sized to carry enough work to hide
// its signalling.  The tasks form one queue, ordered by pipeline depth, so a
// task only ever depends on earlier tasks.
//
// Instances are spread over one queue per XCD (the MI355X has 8 XCDs, each
// with its own L2), balancing estimated cost; all tasks of an instance sit in
// one queue, except for an instance costing more than an eighth of the batch
// (a batch of one), whose tasks are dealt over all queues in turn.  Each
// queue is ordered by pipeline depth.  One persistent kernel of one-wavefront workgroups (as many as
// are resident, rounded down to equal numbers per SIMD) reads the XCD it runs on from the XCC_ID hardware register
// and claims tasks of that XCD's queue with an atomic counter, so an
// instance's data stays near one L2.  A task of stage s of instance p waits
// until p's completion counter reaches the number of p's tasks in stages
// before s (agent-scope acquire), runs, then increments the counter
// (agent-scope release).  The fences are agent-scope because narrower ones
// are not enough: an L1-only invalidation on acquire and a plain store wait
// on release gave wrong results; they also make a dealt instance's results
// visible across XCDs.  No deadlock: a task depends only on tasks of smaller
// depth, and every queue is claimed in depth order by running wavefronts (each
// XCD has resident ones), so an unfinished task of the smallest depth is
// either running with all its inputs done or is reached by its queue once the
// claimed tasks before it, of the same depth, finish.
// A bounded spin turns any unexpected wait into an error flag, not a hang.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mdpe.h"
#include "conv_core.hpp"
#include "plan.hpp"
#include "runtime.hpp"

namespace mdpe {

struct BatchInst {
    double *A;
    const double *coeff;
    const double *z;
    double *value;
    double *grad;
    const int4 *conv;
    const int2 *add;
    const int2 *stage;
    const int *out;
    const int *chains;
    int stride, steps, J;
    int simple;  // deal coefficients to lanes in turn (see conv_group)
    int m, d, n, N;
};

struct BatchTask {
    int inst;
    int kind;   // 0 stage, 1 conv, 2 add, 3 gather
    int need;   // wait until the instance's completion counter reaches this
    int count;  // conv: jobs; others: items (coefficients)
    long first; // conv: first job; add: first (pair, coefficient) item; stage/gather: first item
};

constexpr int kSpinLimit = 1 << 22;
constexpr int kQueues = 8;  // one task queue per XCD

// the XCD (XCC) this wavefront runs on
__device__ __forceinline__ int xcd_id() { return (int)(__builtin_amdgcn_s_getreg(20 | (15 << 11)) & (kQueues - 1)); }

template <int M>
__device__ void run_task(const BatchTask &T, const BatchInst &I, double *lds, int lane) {
    const int d1 = I.d + 1;
    const int kind = __builtin_amdgcn_readfirstlane(T.kind);
    if (kind == 1) {
        for (int g = 0; g < T.count; g += I.J) {
            // chain codes loaded every step: 1.4% faster here (512 mixed
            // instances) than at chain starts
            conv_group<M, false, false, false, true>(I.A, I.conv + T.first + g, min(I.J, T.count - g), I.J, I.d, lds,
                                                     I.chains, I.stride, I.steps, lane, lane, I.simple != 0);
            __syncthreads();
        }
    } else {
        // item T.first + q, q = lane, lane + 64, ...: series e, coefficient c.
        // One 64-bit division per lane and task; each iteration then adds
        // (64 / d1, 64 % d1) with a carry.
        const long f = T.first + lane;
        long e = f / d1;
        int c = (int)(f - e * d1);
        const int qe = 64 / d1, qc = 64 - qe * d1;
        for (int q = lane; q < T.count; q += 64) {
            if (kind == 0)
                stage_item(I.A, I.coeff, I.z, I.stage[e], c, I.N, I.n, I.d, M);
            else if (kind == 2)
                add_item<M>(I.A, I.add[e], c, I.d);
            else
                gather_item(I.A, I.value, I.grad, I.out[e], (int)e, c, I.n, I.d, M);
            e += qe;
            c += qc;
            if (c >= d1) {
                c -= d1;
                ++e;
            }
        }
    }
}

__global__ __launch_bounds__(64) void batch_reset_kernel(int *ctl, int n) {
    for (int i = threadIdx.x; i < n; i += 64) ctl[i] = 0;
}

// ctl[q] = next task of queue q, ctl[kQueues] = error flag,
// ctl[kQueues + 1 + p] = completion counter of instance p.
// qinfo[q] = first task of queue q, qinfo[kQueues + q] = its task count.
// Up to quad double the kernel asks for six resident wavefronts per SIMD
// (at most 80 VGPRs, no spills), the occupancy its register use allowed
// before the convolution loop kept operand addresses per lane.
template <int M1, int M2>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(M2 <= 4 ? 6 : 1))) void batch_kernel(const BatchTask *__restrict__ tasks, const int *__restrict__ qinfo,
                                                   const BatchInst *__restrict__ insts, int *ctl) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int q = xcd_id();
    const int qbase = qinfo[q], qcount = qinfo[kQueues + q];
    int *next = ctl + q, *err = ctl + kQueues, *done = ctl + kQueues + 1;
    // Every value that steers control flow is made wave-uniform (scalar), so
    // the task loop is one scalar loop, never a per-lane divergent one.
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(next, 1);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
        if (t >= qcount) break;
        const BatchTask T = tasks[qbase + t];
        const int inst = __builtin_amdgcn_readfirstlane(T.inst);
        const int need = __builtin_amdgcn_readfirstlane(T.need);
        if (need > 0) {
            // poll without invalidating caches, then one acquire fence
            int spins = 0, ok = 1;
            for (;;) {
                const int v = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(done + inst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                if (v >= need) break;
                const int e = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                if (e || ++spins > kSpinLimit) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(32);  // ~2000 cycles: little polling traffic, small against a task
            }
            if (!ok) {
                if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        const BatchInst I = insts[inst];
        if (__builtin_amdgcn_readfirstlane(I.m) == M1)
            run_task<M1>(T, I, lds, lane);
        else
            run_task<M2>(T, I, lds, lane);
        // release: the fence waits for this wavefront's stores and writes the
        // L2 back; then lane 0 moves the instance's completion counter
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_fetch_add(done + inst, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace mdpe

// ------------------------------------------------------------------ runtime

namespace {

int bfail(int code, const std::string &msg) {
    mdpe::set_last_error(msg);
    return code;
}

#define BHIP(call)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return bfail(MDPE_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

struct mdpe_batch {
    int device = -1;
    int count = 0;
    std::vector<mdpe::BatchInst> insts;
    std::vector<mdpe::BatchTask> tasks;
    mdpe::BatchInst *d_insts = nullptr;
    mdpe::BatchTask *d_tasks = nullptr;
    int *d_qinfo = nullptr;
    int *d_ctl = nullptr;
    std::vector<int> qinfo;      // [2 * kQueues]: first task, task count per queue
    std::vector<int> inst_queue; // queue of each instance, -1: dealt over all queues
    std::vector<int> task_queue; // queue of each task, in task order
    std::vector<int *> d_chains;
    size_t lds = 0;
    int grid = 0;
    bool grid_fixed = false;
    int m1 = 0, m2 = 0;
    bool buffers_set = false;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap = nullptr;
    std::vector<int> stage_tasks;  // tasks per kind, for batch_info
    // eval_and_diff_batch: instance p's workspace starts ws_off[p] bytes into
    // the caller's one workspace of ws_bytes; pointer tables are staged in a
    // ring of pinned host buffers, each reused once its copy has run
    std::vector<int64_t> ws_off;
    int64_t ws_bytes = 0;
    static constexpr int kRing = 4;
    mdpe::BatchInst *ring[kRing] = {};
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    int ring_next = 0;
};

namespace {

void free_batch(mdpe_batch *b) {
    if (!b) return;
    if (b->device < 0) {
        delete b;
        return;
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int r = 0; r < mdpe_batch::kRing; ++r) {
        if (b->ring_ev[r]) {
            (void)hipEventSynchronize(b->ring_ev[r]);
            (void)hipEventDestroy(b->ring_ev[r]);
        }
        if (b->ring[r]) (void)hipHostFree(b->ring[r]);
    }
    (void)hipFree(b->d_insts);
    (void)hipFree(b->d_tasks);
    (void)hipFree(b->d_qinfo);
    (void)hipFree(b->d_ctl);
    for (auto p : b->d_chains) (void)hipFree(p);
    if (prev >= 0 && b->device >= 0) (void)hipSetDevice(prev);
    delete b;
}

// Kernel attributes and the persistent grid (resident one-wavefront
// workgroups), resolved once, outside any stream capture.
template <int M1, int M2>
int prepare_batch(mdpe_batch *b) {
    // the LDS limit is a per-device function attribute: raise it once per device
    static std::atomic<bool> attr[kMaxDevices];
    const int dv = b->device >= 0 && b->device < kMaxDevices ? b->device : 0;
    if (b->lds > 65536 && !attr[dv].load()) {
        BHIP(hipFuncSetAttribute((const void *)mdpe::batch_kernel<M1, M2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)mdpe::kMaxLdsBytes));
        attr[dv].store(true);
    }
    if (b->grid == 0) {
        int per_cu = 0, cus = 0;
        BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)mdpe::batch_kernel<M1, M2>, 64,
                                                          b->lds));
        BHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
        // every XCD needs resident wavefronts to drain its queue; a CU's four
        // SIMDs get equal numbers (17 resident per CU put five on one SIMD,
        // whose tasks ran slowest: 16 measured 0.6% faster on the mixed batch)
        if (per_cu > 4) per_cu -= per_cu % 4;
        b->grid = std::max(1, per_cu) * cus;
    }
    return MDPE_OK;
}

template <int M1, int M2>
int launch_batch(mdpe_batch *b, hipStream_t st, bool prepare_only) {
    int rc = prepare_batch<M1, M2>(b);
    if (rc || prepare_only) return rc;
    hipLaunchKernelGGL(mdpe::batch_reset_kernel, dim3(1), dim3(64), 0, st, b->d_ctl, b->count + mdpe::kQueues + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(MDPE_EDEVICE, std::string("batch_reset_kernel: ") + hipGetErrorString(e));
    hipLaunchKernelGGL((mdpe::batch_kernel<M1, M2>), dim3(b->grid), dim3(64), b->lds, st, b->d_tasks, b->d_qinfo,
                       b->d_insts, b->d_ctl);
    e = hipGetLastError();
    if (e != hipSuccess) return bfail(MDPE_EDEVICE, std::string("batch_kernel: ") + hipGetErrorString(e));
    return MDPE_OK;
}

int launch_any(mdpe_batch *b, hipStream_t st, bool prepare_only = false) {
#define MS(a, c) (b->m1 == (a) && b->m2 == (c))
    if (MS(1, 1)) return launch_batch<1, 1>(b, st, prepare_only);
    if (MS(2, 2)) return launch_batch<2, 2>(b, st, prepare_only);
    if (MS(3, 3)) return launch_batch<3, 3>(b, st, prepare_only);
    if (MS(4, 4)) return launch_batch<4, 4>(b, st, prepare_only);
    if (MS(5, 5)) return launch_batch<5, 5>(b, st, prepare_only);
    if (MS(8, 8)) return launch_batch<8, 8>(b, st, prepare_only);
    if (MS(10, 10)) return launch_batch<10, 10>(b, st, prepare_only);
    if (MS(2, 4)) return launch_batch<2, 4>(b, st, prepare_only);
#undef MS
    return bfail(MDPE_EUNSUPPORTED, "batch precisions must be all equal, or {2, 4}");
}

// ------------------------------------------------------- the tune cache --
// The autotuner writes JSON: {"<arch>": {"tiles": [{"m": .., "d": ..,
// "jobs_per_group": .., "groups_per_task": .., "add_items_per_task": ..}, ...],
// other keys ...}, ...}.  A small reader for exactly that much JSON.
struct JVal {
    enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal *get(const std::string &k) const {
        for (auto &kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct JReader {
    const char *p, *e;
    void ws() {
        while (p < e && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool lit(const char *w) {
        const size_t n = std::strlen(w);
        if ((size_t)(e - p) < n || std::strncmp(p, w, n) != 0) return false;
        p += n;
        return true;
    }
    bool string(std::string &out) {
        if (p >= e || *p != '"') return false;
        for (++p; p < e && *p != '"'; ++p) {
            if (*p == '\\') {
                if (++p >= e) return false;
                out.push_back(*p == 'n' ? '\n' : *p == 't' ? '\t' : *p);  // \uXXXX is not expected in a tune cache
            } else {
                out.push_back(*p);
            }
        }
        if (p >= e) return false;
        ++p;
        return true;
    }
    bool value(JVal &v, int depth) {
        if (depth > 32) return false;
        ws();
        if (p >= e) return false;
        if (*p == '{') {
            v.kind = JVal::kObj;
            ++p;
            ws();
            if (p < e && *p == '}') return ++p, true;
            for (;;) {
                ws();
                std::string k;
                if (!string(k)) return false;
                ws();
                if (p >= e || *p++ != ':') return false;
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.obj.emplace_back(std::move(k), std::move(x));
                ws();
                if (p < e && *p == ',') { ++p; continue; }
                if (p < e && *p == '}') return ++p, true;
                return false;
            }
        }
        if (*p == '[') {
            v.kind = JVal::kArr;
            ++p;
            ws();
            if (p < e && *p == ']') return ++p, true;
            for (;;) {
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.arr.push_back(std::move(x));
                ws();
                if (p < e && *p == ',') { ++p; continue; }
                if (p < e && *p == ']') return ++p, true;
                return false;
            }
        }
        if (*p == '"') {
            v.kind = JVal::kStr;
            return string(v.str);
        }
        if (lit("true") || lit("false")) return v.kind = JVal::kBool, true;
        if (lit("null")) return true;
        char *end = nullptr;
        std::string num(p, (size_t)std::min<ptrdiff_t>(e - p, 64));
        v.num = std::strtod(num.c_str(), &end);
        if (end == num.c_str()) return false;
        v.kind = JVal::kNum;
        p += end - num.c_str();
        return true;
    }
};

// Tiles for `arch` from the cache file at `path`; an absent arch key gives
// no tiles (the defaults).  Returns "" or an error message.
std::string read_tune_cache(const char *path, const std::string &arch, std::vector<mdpe_batch_tile> &tiles) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return std::string("cannot read the tune cache ") + path;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, got);
        if (text.size() > (16u << 20)) break;
    }
    std::fclose(f);
    JVal root;
    JReader r{text.data(), text.data() + text.size()};
    if (!r.value(root, 0) || root.kind != JVal::kObj) return std::string("tune cache ") + path + ": not a JSON object";
    const JVal *dev = root.get(arch);
    if (!dev) return "";
    const JVal *list = dev->kind == JVal::kObj ? dev->get("tiles") : nullptr;
    if (!list || list->kind != JVal::kArr) return std::string("tune cache ") + path + ": no tile list for " + arch;
    for (const JVal &t : list->arr) {
        auto field = [&](const char *k, bool need, int32_t &out) {
            const JVal *x = t.kind == JVal::kObj ? t.get(k) : nullptr;
            if (!x) return !need;
            if (x->kind != JVal::kNum || x->num < 0 || x->num > 1e9 || x->num != (double)(int64_t)x->num) return false;
            out = (int32_t)x->num;
            return true;
        };
        mdpe_batch_tile tile{0, 0, 0, 0, 0, 0};
        if (!field("m", true, tile.m) || !field("d", true, tile.d) || !field("jobs_per_group", false, tile.jobs_per_group) ||
            !field("groups_per_task", false, tile.groups_per_task) ||
            !field("add_items_per_task", false, tile.add_items_per_task) || !field("deal", false, tile.deal) ||
            tile.deal > 2)
            return std::string("tune cache ") + path + ": a tile needs integer m, d and tile fields (deal 0, 1 or 2)";
        tiles.push_back(tile);
    }
    return "";
}

// the device's architecture name without feature suffixes ("gfx950")
std::string device_arch(int device) {
    hipDeviceProp_t prop;
    if (device < 0 || hipGetDeviceProperties(&prop, device) != hipSuccess) return "gfx950";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// capture [reset, persistent kernel] once on a private stream, replay on `stream`
int launch_graph_on(mdpe_batch *b, hipStream_t stream) {
    int rc = MDPE_OK;
    if (!b->exec) {
        if (!b->cap) BHIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        rc = launch_any(b, b->cap, true);  // attributes and grid, outside the capture
        if (!rc) {
            BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
            rc = launch_any(b, b->cap);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->cap, &g);
            if (!rc && e != hipSuccess) rc = bfail(MDPE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            if (!rc) {
                b->graph = g;
                e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) rc = bfail(MDPE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
    }
    if (!rc) {
        hipError_t e = hipGraphLaunch(b->exec, stream);
        if (e != hipSuccess) rc = bfail(MDPE_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    }
    return rc;
}

}  // namespace

extern "C" {

int plan_batch(const mdpe_plan *const *plans, int count, const char *tune_cache, mdpe_batch **out) {
    if (!plans || !out || count <= 0) return bfail(MDPE_EINVAL, "plans, count > 0 and out are required");
    *out = nullptr;
    std::vector<mdpe_batch_tile> tiles;
    if (tune_cache && *tune_cache) {
        if (!plans[0]) return bfail(MDPE_EINVAL, "NULL plan in the batch");
        std::string err;
        try {
            err = read_tune_cache(tune_cache, device_arch(plans[0]->device), tiles);
        } catch (const std::bad_alloc &) {
            return bfail(MDPE_ENOMEM, "host allocation failed while reading the tune cache");
        }
        if (!err.empty()) return bfail(MDPE_EINVAL, err);
    }
    return plan_batch_tiles(plans, count, tiles.data(), (int)tiles.size(), out);
}

int plan_batch_tiles(const mdpe_plan *const *plans, int count, const mdpe_batch_tile *tiles, int ntiles,
                     mdpe_batch **out) {
    if (!plans || !out || count <= 0) return bfail(MDPE_EINVAL, "plans, count > 0 and out are required");
    if (ntiles < 0 || (ntiles > 0 && !tiles)) return bfail(MDPE_EINVAL, "bad tiles");
    for (int q = 0; q < ntiles; ++q)
        if (tiles[q].deal < 0 || tiles[q].deal > 2) return bfail(MDPE_EINVAL, "a tile's deal must be 0, 1 or 2");
    *out = nullptr;
    std::unique_ptr<mdpe_batch> B(new (std::nothrow) mdpe_batch());
    if (!B) return bfail(MDPE_ENOMEM, "host allocation failed");
    B->count = count;
    std::vector<int> ms;
    for (int p = 0; p < count; ++p) {
        if (!plans[p]) return bfail(MDPE_EINVAL, "NULL plan in the batch");
        const mdpe::Plan *P = &plans[p]->P;
        int dev = plans[p]->device;
        if (p == 0) B->device = dev;
        if (dev != B->device) return bfail(MDPE_EINVAL, "plans on different devices (or host-only mixed in)");
        if (P->complex_series()) return bfail(MDPE_EUNSUPPORTED, "batches hold real series only (MDPE_COMPLEX plan)");
        if (!P->scale.empty()) return bfail(MDPE_EUNSUPPORTED, "batches hold multilinear polynomials only (exponents)");
        if (P->streamed) return bfail(MDPE_EUNSUPPORTED, "batches stage operands in LDS (streamed-operand plan)");
        if (std::find(ms.begin(), ms.end(), P->m) == ms.end()) ms.push_back(P->m);
    }
    std::sort(ms.begin(), ms.end());
    if (ms.size() == 1) {
        B->m1 = B->m2 = ms[0];
    } else if (ms.size() == 2 && ms[0] == 2 && ms[1] == 4) {
        B->m1 = 2;
        B->m2 = 4;
    } else {
        return bfail(MDPE_EUNSUPPORTED, "batch precisions must be all equal, or {2, 4}");
    }
    auto tile_for = [&](int m, int d) {
        mdpe_batch_tile t{m, d, 0, 0, 0, 0};
        for (int q = 0; q < ntiles; ++q)
            if (tiles[q].m == m && tiles[q].d == d) t = tiles[q];
        if (t.jobs_per_group <= 0) t.jobs_per_group = mdpe::choose_jobs_per_group(d, m);
        return t;
    };
    // schedules per (d, J)
    std::map<std::pair<int, int>, int> sched_index;
    std::vector<mdpe::LaneSchedule> scheds;
    // tasks with their depth and an instance cost for ordering
    struct Tmp {
        int queue;
        int depth;
        double cost;
        int order;
        mdpe::BatchTask t;
    };
    // estimated cost per instance (multiply-adds x limbs^2), then longest-first
    // assignment of instances to the XCD queues
    std::vector<double> icost(count);
    for (int p = 0; p < count; ++p) {
        const mdpe::Plan &P = plans[p]->P;
        const double d1 = P.d + 1;
        icost[p] = ((double)P.conv.size() * d1 * (d1 + 1) / 2 + (double)P.add.size() * d1) * P.m * P.m + d1;
    }
    std::vector<int> order_p(count);
    for (int p = 0; p < count; ++p) order_p[p] = p;
    std::stable_sort(order_p.begin(), order_p.end(), [&](int a, int c) { return icost[a] > icost[c]; });
    // An instance costing more than one queue's fair share (a batch of one, or
    // a few large instances) has its tasks dealt over all queues in turn, so it
    // runs on every XCD; the others keep one queue each, near one L2.
    double total = 0;
    for (double c : icost) total += c;
    std::vector<double> qload(mdpe::kQueues, 0.0);
    B->inst_queue.assign(count, 0);
    for (int p : order_p)
        if (icost[p] > total / mdpe::kQueues) {
            B->inst_queue[p] = -1;
            for (auto &l : qload) l += icost[p] / mdpe::kQueues;
        }
    for (int p : order_p) {
        if (B->inst_queue[p] < 0) continue;
        int best = 0;
        for (int q = 1; q < mdpe::kQueues; ++q)
            if (qload[q] < qload[best]) best = q;
        qload[best] += icost[p];
        B->inst_queue[p] = best;
    }
    std::vector<Tmp> tmp;
    B->insts.resize(count);
    // one workspace for all instances: each instance's part 256-byte aligned
    B->ws_off.resize(count);
    for (int p = 0; p < count; ++p) {
        const mdpe::Plan &P = plans[p]->P;
        B->ws_off[p] = B->ws_bytes;
        const int64_t bytes = P.n_series * (int64_t)(P.d + 1) * P.w * (int64_t)sizeof(double);
        B->ws_bytes += (bytes + 255) / 256 * 256;
    }
    size_t lds = 0;
    for (int p = 0; p < count; ++p) {
        const mdpe::Plan &P = plans[p]->P;
        const mdpe_batch_tile t = tile_for(P.m, P.d);
        const int J = t.jobs_per_group;
        auto key = std::make_pair(P.d, J);
        if (!sched_index.count(key)) {
            sched_index[key] = (int)scheds.size();
            scheds.push_back(mdpe::make_lane_schedule(P.d, J));
        }
        const mdpe::LaneSchedule &S = scheds[sched_index[key]];
        // a dealt instance finds its parallelism inside its own layers: one
        // group of jobs per task, small addition tasks
        const bool dealt = B->inst_queue[p] < 0;
        const int G = dealt ? 1 : t.groups_per_task > 0 ? t.groups_per_task : std::max(1, (256 + S.steps - 1) / S.steps);
        const long items_per_task = dealt ? 1024 : t.add_items_per_task > 0 ? t.add_items_per_task : 4096;
        lds = std::max(lds, (size_t)mdpe::group_lds_bytes(P.d + 1, mdpe::lds_doubles_per_coef(P.m), J));
        if (lds > (size_t)mdpe::kMaxLdsBytes)
            return bfail(MDPE_EUNSUPPORTED, "a tile's jobs_per_group needs more LDS than one workgroup has");
        mdpe::BatchInst &I = B->insts[p];
        std::memset(&I, 0, sizeof(I));
        I.conv = plans[p]->d_conv;
        I.add = plans[p]->d_add;
        I.stage = plans[p]->d_stage;
        I.out = plans[p]->d_out;
        I.stride = S.stride;
        I.steps = S.steps;
        I.J = J;
        I.simple = P.m > 2 ? 0 : t.deal == 1 ? 0 : t.deal == 2 ? 1 : mdpe::prefer_simple_dealing(P.d, J, P.m, S.steps) ? 1 : 0;
        I.m = P.m;
        I.d = P.d;
        I.n = P.n;
        I.N = P.N;
        const int d1 = P.d + 1;
        const double cost = icost[p];
        const int queue = B->inst_queue[p];
        int depth = 0, done_before = 0, order = 0;
        auto emit = [&](int kind, long first, int cnt, int need) {
            const int q = queue >= 0 ? queue : (p + order) % mdpe::kQueues;
            tmp.push_back({q, depth, cost, order++, {p, kind, need, cnt, first}});
        };
        auto items = [&](int kind, long total) {
            int n = 0;
            for (long f = 0; f < total; f += items_per_task, ++n)
                emit(kind, f, (int)std::min(items_per_task, total - f), done_before);
            return n;
        };
        // stage
        done_before += items(0, (long)P.stage.size() * d1);
        ++depth;
        for (int L = 1; L <= P.n_layers(); ++L, ++depth) {
            const long a = P.conv_off[L - 1], z = P.conv_off[L];
            int n = 0;
            for (long f = a; f < z; f += (long)G * J, ++n) emit(1, f, (int)std::min((long)G * J, z - f), done_before);
            done_before += n;
        }
        for (int r = 1; r <= P.n_levels(); ++r, ++depth) {
            const long a = P.add_off[r - 1] * d1, z = P.add_off[r] * d1;
            int n = 0;
            for (long f = a; f < z; f += items_per_task, ++n)
                emit(2, f, (int)std::min(items_per_task, z - f), done_before);
            done_before += n;
        }
        done_before += items(3, (long)(1 + P.n) * d1);
    }
    std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp &a, const Tmp &b) {
        if (a.queue != b.queue) return a.queue < b.queue;
        if (a.depth != b.depth) return a.depth < b.depth;
        if (a.cost != b.cost) return a.cost > b.cost;
        if (a.t.inst != b.t.inst) return a.t.inst < b.t.inst;
        return a.order < b.order;
    });
    B->qinfo.assign(2 * mdpe::kQueues, 0);
    for (size_t q = 0; q < tmp.size(); ++q) {
        B->tasks.push_back(tmp[q].t);
        B->task_queue.push_back(tmp[q].queue);
        B->qinfo[mdpe::kQueues + tmp[q].queue]++;
    }
    for (int q = 1; q < mdpe::kQueues; ++q) B->qinfo[q] = B->qinfo[q - 1] + B->qinfo[mdpe::kQueues + q - 1];
    B->lds = lds;
    B->stage_tasks.assign(4, 0);
    for (auto &t : B->tasks) B->stage_tasks[t.kind]++;
    if (B->device < 0) {  // host-only batch: for inspecting the queue
        *out = B.release();
        return MDPE_OK;
    }
    // device arrays
    int prev = -1;
    (void)hipGetDevice(&prev);
    BHIP(hipSetDevice(B->device));
    int rc = MDPE_OK;
    auto alloc_copy = [&](void **dst, const void *src, size_t bytes) -> int {
        BHIP(hipMalloc(dst, bytes ? bytes : 16));
        if (bytes) BHIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return MDPE_OK;
    };
    for (auto &S : scheds) {
        int *dc = nullptr;
        if ((rc = alloc_copy((void **)&dc, S.chains.data(), S.chains.size() * sizeof(int)))) break;
        B->d_chains.push_back(dc);
    }
    if (!rc) {
        for (int p = 0; p < count; ++p) {
            const mdpe::Plan &P = plans[p]->P;
            B->insts[p].chains = B->d_chains[sched_index[{P.d, B->insts[p].J}]];
        }
        if (!(rc = alloc_copy((void **)&B->d_tasks, B->tasks.data(), B->tasks.size() * sizeof(mdpe::BatchTask))) &&
            !(rc = alloc_copy((void **)&B->d_qinfo, B->qinfo.data(), B->qinfo.size() * sizeof(int))))
            if (!(rc = alloc_copy((void **)&B->d_insts, B->insts.data(), B->insts.size() * sizeof(mdpe::BatchInst)))) {
                // control words: zeroed by the reset kernel before every launch
                hipError_t e = hipMalloc((void **)&B->d_ctl, sizeof(int) * (size_t)(count + mdpe::kQueues + 1));
                if (e != hipSuccess) rc = bfail(MDPE_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
            }
    }
    for (int r = 0; !rc && r < mdpe_batch::kRing; ++r) {
        hipError_t e = hipHostMalloc((void **)&B->ring[r], sizeof(mdpe::BatchInst) * (size_t)count, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ring_ev[r], hipEventDisableTiming);
        if (e != hipSuccess) rc = bfail(MDPE_EDEVICE, std::string("pinned pointer tables: ") + hipGetErrorString(e));
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    if (rc) {
        std::string keep = mdpe::get_last_error();
        free_batch(B.release());
        mdpe::set_last_error(keep);
        return rc;
    }
    *out = B.release();
    return MDPE_OK;
}

int batch_info(const mdpe_batch *b, mdpe_batch_info *o) {
    if (!b || !o) return bfail(MDPE_EINVAL, "batch and out are required");
    o->count = b->count;
    o->n_tasks = (int64_t)b->tasks.size();
    o->n_conv_tasks = b->stage_tasks[1];
    o->n_add_tasks = b->stage_tasks[2];
    o->lds_bytes = (int64_t)b->lds;
    o->grid = b->grid;
    o->m1 = b->m1;
    o->m2 = b->m2;
    o->workspace_bytes = b->ws_bytes;
    return MDPE_OK;
}

int batch_tasks(const mdpe_batch *b, int32_t *rows) {
    if (!b || !rows) return bfail(MDPE_EINVAL, "batch and rows are required");
    for (size_t q = 0; q < b->tasks.size(); ++q) {
        const auto &t = b->tasks[q];
        rows[6 * q] = t.inst;
        rows[6 * q + 1] = t.kind;
        rows[6 * q + 2] = t.need;
        rows[6 * q + 3] = t.count;
        rows[6 * q + 4] = (int32_t)t.first;
        rows[6 * q + 5] = b->task_queue[q];
    }
    return MDPE_OK;
}

int batch_set_buffers(mdpe_batch *b, const double *const *coeff, const double *const *z, double *const *value,
                      double *const *grad, void *const *workspace) {
    if (!b || !coeff || !z || !value || !grad || !workspace) return bfail(MDPE_EINVAL, "NULL argument");
    if (b->device < 0) return bfail(MDPE_EINVAL, "host-only batch");
    for (int p = 0; p < b->count; ++p) {
        if (!coeff[p] || !z[p] || !value[p] || !grad[p] || !workspace[p])
            return bfail(MDPE_EINVAL, "NULL buffer for instance " + std::to_string(p));
        if (((uintptr_t)workspace[p]) % 256) return bfail(MDPE_EINVAL, "workspace must be 256-byte aligned");
        b->insts[p].A = (double *)workspace[p];
        b->insts[p].coeff = coeff[p];
        b->insts[p].z = z[p];
        b->insts[p].value = value[p];
        b->insts[p].grad = grad[p];
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    BHIP(hipSetDevice(b->device));
    hipError_t e = hipMemcpy(b->d_insts, b->insts.data(), b->insts.size() * sizeof(mdpe::BatchInst),
                             hipMemcpyHostToDevice);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) return bfail(MDPE_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    b->buffers_set = true;
    return MDPE_OK;
}

int batch_launch(mdpe_batch *b, void *stream) {
    if (!b) return bfail(MDPE_EINVAL, "batch is NULL");
    if (!b->buffers_set) return bfail(MDPE_EINVAL, "call batch_set_buffers first");
    int prev = -1;
    (void)hipGetDevice(&prev);
    BHIP(hipSetDevice(b->device));
    int rc = launch_any(b, (hipStream_t)stream);
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
}

int batch_launch_graph(mdpe_batch *b, void *stream) {
    if (!b) return bfail(MDPE_EINVAL, "batch is NULL");
    if (!b->buffers_set) return bfail(MDPE_EINVAL, "call batch_set_buffers first");
    int prev = -1;
    (void)hipGetDevice(&prev);
    BHIP(hipSetDevice(b->device));
    int rc = launch_graph_on(b, (hipStream_t)stream);
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
}

int eval_and_diff_batch(mdpe_batch *b, const double *const *coeff, const double *const *z, double *const *value,
                        double *const *grad, void *workspace, void *stream) {
    if (!b || !coeff || !z || !value || !grad || !workspace) return bfail(MDPE_EINVAL, "NULL argument");
    if (b->device < 0) return bfail(MDPE_EINVAL, "host-only batch");
    if (((uintptr_t)workspace) % 256) return bfail(MDPE_EINVAL, "workspace must be 256-byte aligned");
    bool changed = !b->buffers_set;
    for (int p = 0; p < b->count; ++p) {
        if (!coeff[p] || !z[p] || !value[p] || !grad[p])
            return bfail(MDPE_EINVAL, "NULL buffer for instance " + std::to_string(p));
    }
    for (int p = 0; p < b->count; ++p) {
        mdpe::BatchInst &I = b->insts[p];
        double *A = (double *)((char *)workspace + b->ws_off[p]);
        changed |= I.A != A || I.coeff != coeff[p] || I.z != z[p] || I.value != value[p] || I.grad != grad[p];
        I.A = A;
        I.coeff = coeff[p];
        I.z = z[p];
        I.value = value[p];
        I.grad = grad[p];
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    BHIP(hipSetDevice(b->device));
    hipStream_t st = (hipStream_t)stream;
    int rc = MDPE_OK;
    if (changed) {
        // stream-ordered rebinding: the table goes through a pinned buffer
        // whose previous copy (kRing rebinds ago) has run by now, unless the
        // caller is more than kRing rebinds ahead of the device
        const int r = b->ring_next;
        b->ring_next = (r + 1) % mdpe_batch::kRing;
        hipError_t e = b->ring_used[r] ? hipEventSynchronize(b->ring_ev[r]) : hipSuccess;
        if (e == hipSuccess) {
            std::memcpy(b->ring[r], b->insts.data(), sizeof(mdpe::BatchInst) * (size_t)b->count);
            e = hipMemcpyAsync(b->d_insts, b->ring[r], sizeof(mdpe::BatchInst) * (size_t)b->count,
                               hipMemcpyHostToDevice, st);
        }
        if (e == hipSuccess) e = hipEventRecord(b->ring_ev[r], st);
        if (e != hipSuccess) rc = bfail(MDPE_EDEVICE, std::string("binding the pointer table: ") + hipGetErrorString(e));
        b->ring_used[r] = true;
        b->buffers_set = !rc;
    }
    if (!rc) rc = launch_graph_on(b, st);
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
}

int batch_status(mdpe_batch *b) {
    if (!b) return bfail(MDPE_EINVAL, "batch is NULL");
    if (b->device < 0) return bfail(MDPE_EINVAL, "host-only batch");
    int flags[mdpe::kQueues + 1] = {0};
    int prev = -1;
    (void)hipGetDevice(&prev);
    BHIP(hipSetDevice(b->device));
    BHIP(hipDeviceSynchronize());
    hipError_t e = hipMemcpy(flags, b->d_ctl, sizeof(flags), hipMemcpyDeviceToHost);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) return bfail(MDPE_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    if (flags[mdpe::kQueues]) return bfail(MDPE_EDEVICE, "batch watchdog: a task waited too long for its inputs");
    for (int q = 0; q < mdpe::kQueues; ++q)
        if (flags[q] < b->qinfo[mdpe::kQueues + q])
            return bfail(MDPE_EDEVICE, "batch queue " + std::to_string(q) + " was not drained (no wavefront ran on its XCD)");
    return MDPE_OK;
}

int batch_set_grid(mdpe_batch *b, int grid) {
    if (!b || grid < 0) return bfail(MDPE_EINVAL, "batch is NULL or grid < 0");
    if (b->exec) return bfail(MDPE_EINVAL, "the batch's graph is already captured");
    b->grid = grid;  // 0: resident capacity, resolved at the next launch
    b->grid_fixed = grid > 0;
    return MDPE_OK;
}

void batch_destroy(mdpe_batch *b) { free_batch(b); }

}  // extern "C"
