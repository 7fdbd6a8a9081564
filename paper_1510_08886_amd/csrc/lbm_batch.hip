// Batched and served channel solves (2D, nx = 1): many independent plane
// Poiseuille channels, each stepped by one workgroup with its populations in
// LDS, each run to a steady-state tolerance on the mass flow.
//
// Device side: k_slots walks a list of resident slots (one workgroup per slot
// in the served mode, or a device work queue in the persistent mode). For its
// slot a workgroup loads the stored populations ([alpha][y], storage type) into
// LDS and steps: gather the pull sources of its rows from LDS, patch the wall
// slots, collide, then (after a barrier) store the rows back and the FP64
// wall-flux partials. The per-node arithmetic is the one of the HBM step kernel
// (lbm_node2d.h), stochastic-rounding keys included, and the mass-flow test is
// the one of lbm_run_to_tol, with a fixed-shape FP64 tree over the rows, so a
// channel's result depends neither on the workgroup size nor on its neighbours.
//
// Host side: a slot table and a first-fit allocator over the caller's pool;
// requests are admitted when a slot and their state bytes are free; each
// served launch advances every resident channel by a quantum of steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <type_traits>
#include <vector>

#include "lbm_node2d.h"

namespace lbm {

enum SlotStatus : int { kRunning = 0, kConverged = 1, kCapped = 2, kFailed = 3 };

// Sets the batched kernel is compiled for (index = SET::ID).
constexpr int kBatchSets = 2;   // D2V17, D2V37

struct SlotDesc {
    int set;             // SetD2V17::ID or SetD2V37::ID
    int ny;
    int check_every;
    int status;          // SlotStatus
    int fresh;           // 1: start from the rest state rho0 w
    int have_prev;
    double tol;
    int64_t max_steps;
    int64_t steps;
    double mdot, mdot_prev;
    double mdot_scale;
    uint64_t pop_off;    // byte offset of the stored populations in the pool
    double apart[2][4];  // FP64 wall-flux partials [face][row]
    StepScalars<float> sc;     // FP32 collision
    StepScalars<double> scd;   // FP64 collision (LBM_F32SR)
};

template <typename R>
__device__ __forceinline__ const StepScalars<R> &slot_scalars(const SlotDesc *d) {
    if constexpr (std::is_same<R, double>::value)
        return d->scd;
    else
        return d->sc;
}

// LDS bytes one slot needs: populations, the padded reduction tree, partials
__host__ __device__ inline size_t slot_lds_bytes(int V, int ny, int elem) {
    size_t f = ((size_t)V * ny * elem + 15) / 16 * 16;
    size_t p = 1;
    while ((int)p < ny) p <<= 1;
    return f + p * 8 + 2 * 4 * 8;
}

template <class SET, Storage S, int RMAX>
__device__ __forceinline__ void run_slot(unsigned char *pool, SlotDesc *d,
                                         const PairTable<typename St<S>::R> &t, unsigned char *lds,
                                         int64_t quantum) {
    using T = typename St<S>::T;
    using R = typename St<S>::R;
    constexpr int V = SET::V, NR = SET::NR, HN = SET::HN;
    const int ny = d->ny;
    const int TH = blockDim.x;
    const StepScalars<R> &s = slot_scalars<R>(d);
    T *f = (T *)lds;
    int P = 1;
    while (P < ny) P <<= 1;
    double *red = (double *)(lds + ((size_t)V * ny * sizeof(T) + 15) / 16 * 16);
    double *ap = red + P;   // [face][row < HN]
    T *g = (T *)(pool + d->pop_off);

    // state into LDS
    if (d->fresh) {
        // rest state rho0 w: deviation 0
        for (int e = threadIdx.x; e < V * ny; e += TH) {
            const int a = e / ny;
            const int p = (a - NR) >> 1;
            T v;
            if (NR && a == 0)
                v = encode_dev<S, false>(R(0), t.wr00, t.inv_wr00, 0);
            else
                v = encode_dev<S, false>(R(0), t.wr0[p], t.inv_wr0[p], 0);
            f[e] = v;
        }
    } else {
        for (int e = threadIdx.x; e < V * ny; e += TH) f[e] = g[e];
    }
    if ((int)threadIdx.x < 2 * HN) ap[threadIdx.x] = d->apart[threadIdx.x / HN][threadIdx.x % HN];
    __syncthreads();

    int64_t steps = d->steps;
    double prev = d->mdot_prev, mdot = d->mdot;
    int have = d->have_prev;
    int status = kRunning;
    const int64_t max_steps = d->max_steps;
    const int ce = d->check_every;
    const double tol = d->tol, mscale = d->mdot_scale;

    for (int64_t q = 0; q < quantum; ++q) {
        R dd[RMAX][V];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int j = threadIdx.x + r * TH;
            if (j < ny) {
                T raw[V];
                if constexpr (NR) raw[0] = f[j];
                for_pairs<SET::NP>([&](auto pc) {
                    constexpr int p = decltype(pc)::value;
                    constexpr int ey = SET::EY[p];
                    const int jp = min(max(j - ey, 0), ny - 1);
                    const int jm = min(max(j + ey, 0), ny - 1);
                    raw[NR + 2 * p] = f[(NR + 2 * p) * ny + jp];
                    raw[NR + 2 * p + 1] = f[(NR + 2 * p + 1) * ny + jm];
                });
                complete2d<SET, S>(raw, ap, t, s, 0, j, dd[r]);
            }
        }
        const bool check = (steps > 0 && steps % ce == 0) || steps >= max_steps;
        if (check) {
            // mass flow of the streamed state: FP64 tree over the padded rows
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                const int j = threadIdx.x + r * TH;
                if (j < ny) red[j] = (double)moments2d<SET, R>(dd[r], s, t.c).ux;
            }
            for (int e = ny + threadIdx.x; e < P; e += TH) red[e] = 0.0;
            __syncthreads();
            for (int h = P >> 1; h > 0; h >>= 1) {
                for (int e = threadIdx.x; e < h; e += TH) red[e] += red[e + h];
                __syncthreads();
            }
            const double md = mscale * red[0] / ny;
            __syncthreads();
            const bool conv = have && fabs(md - prev) < tol * fabs(md);
            mdot = md;
            prev = md;
            have = 1;
            if (!isfinite(md)) {
                status = kFailed;
                break;
            }
            if (conv) {
                status = kConverged;
                break;
            }
        }
        if (steps >= max_steps) {
            status = kCapped;
            break;
        }
        __syncthreads();   // every row has read its sources
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int j = threadIdx.x + r * TH;
            if (j < ny) {
                relax2d<SET, R>(dd[r], t, s, t.c);
                T v[V];
                encode_all<SET, S, true>(dd[r], t, (uint32_t)j, (uint32_t)steps, v);
#pragma unroll
                for (int a = 0; a < V; ++a) f[a * ny + j] = v[a];
                wall_partials2d<SET, S>(v, t, s, 0, j, ap);
            }
        }
        __syncthreads();
        ++steps;
    }
    // state back to the pool
    for (int e = threadIdx.x; e < V * ny; e += TH) g[e] = f[e];
    if ((int)threadIdx.x < 2 * HN) d->apart[threadIdx.x / HN][threadIdx.x % HN] = ap[threadIdx.x];
    if (threadIdx.x == 0) {
        d->steps = steps;
        d->mdot = mdot;
        d->mdot_prev = prev;
        d->have_prev = have;
        d->status = status;
        d->fresh = 0;
    }
    __syncthreads();
}

// counter == nullptr: workgroup b runs slot active[b] for `quantum` steps.
// Otherwise workgroups take slots from the device work queue until it is
// exhausted; every workgroup leaves once the counter passes nactive.
// MAXT is the largest workgroup the instance is launched with: the register
// budget per thread follows from it (1024 threads leave 128 VGPRs, which the
// node state of two rows per thread overflows into scratch memory).
template <Storage S, int RMAX, int MAXT>
__global__ __launch_bounds__(MAXT) void k_slots(unsigned char *pool, SlotDesc *descs,
                                                const void *tab_mem, const int *active,
                                                int nactive, int *counter, int64_t quantum) {
    using R = typename St<S>::R;
    const auto *tabs = (const PairTable<R> *)tab_mem;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int s_idx;
    int k = blockIdx.x;
    for (;;) {
        if (counter) {
            if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
            __syncthreads();
            k = s_idx;
            __syncthreads();
        }
        if (k >= nactive) break;
        SlotDesc *d = descs + active[k];
        if (d->set == SetD2V17::ID)
            run_slot<SetD2V17, S, RMAX>(pool, d, tabs[SetD2V17::ID], lds, quantum);
        else
            run_slot<SetD2V37, S, RMAX>(pool, d, tabs[SetD2V37::ID], lds, quantum);
        if (!counter) break;
    }
}

__global__ void k_reset_counter(int *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// ---------------------------------------------------------------------------
// host engine
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kAl = 256;
size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

struct Req {
    uint64_t id;
    int set;
    int ny;
    double kn;
    double tol;
    int check_every;
    int64_t max_steps;
    double est;          // estimated work (for longest-first ordering)
    uint64_t seq;        // submission order
    StepScalars<float> sc;
    StepScalars<double> scd;
    double mdot_scale;
    double apart0[2][4];
};

}  // namespace

struct Batch {
    int max_slots = 0;
    Storage st = Storage::F32;
    int elem = 4;
    unsigned char *pool = nullptr;
    size_t pool_bytes = 0;
    hipStream_t stream = nullptr;
    size_t off_desc = 0, off_tabs = 0, off_counter = 0, off_active = 0, off_heap = 0;
    SlotDesc *h_desc = nullptr;      // pinned mirror of the slot table
    int *h_active = nullptr;         // pinned active list
    std::vector<int> free_slots;
    std::map<size_t, size_t> free_blocks;   // offset -> bytes (heap region)
    std::deque<Req> queue;
    struct Act {
        int slot;
        Req req;
        size_t off, bytes;
    };
    std::vector<Act> active;
    std::vector<lbm_result_t> done;
    bool tab_set[kBatchSets] = {false, false};
    PairTable<float> tabs[kBatchSets];
    int threads = 512;
    int quantum = 1000;
    int slots_per_cu = 2;            // persistent mode: resident workgroups per CU (LDS permitting)
    int order = LBM_BATCH_LONGEST_FIRST;   // persistent mode: work-queue order
    uint64_t next_seq = 0;
    bool inflight = false;
    // persistent launches captured once per launch shape and replayed
    struct Graph {
        int nact, grid, threads, rmax;
        size_t lds;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    int64_t graph_replays = 0;
    hipEvent_t ev = nullptr;
    int64_t launches = 0;
    size_t max_lds = 65536;
    int cus = 1;
    size_t used = 0;

    size_t heap_free() const {
        size_t t = 0;
        for (auto &kv : free_blocks) t += kv.second;
        return t;
    }
    bool alloc(size_t bytes, size_t &off) {
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_blocks.erase(it);
                if (rest) free_blocks[off + bytes] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        used -= bytes;
        auto it = free_blocks.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_blocks.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_blocks.erase(nx);
        }
        if (it != free_blocks.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_blocks.erase(it);
            }
        }
    }
    int V_of(int set) const { return set == SetD2V17::ID ? SetD2V17::V : SetD2V37::V; }
    size_t state_bytes(const Req &r) const { return al((size_t)V_of(r.set) * r.ny * elem); }
    size_t lds_bytes(const Req &r) const { return slot_lds_bytes(V_of(r.set), r.ny, elem); }
};

static int launch_slots(Batch &b, int nact, bool persistent, int64_t quantum, size_t lds,
                        int rmax, int grid) {
    auto *descs = (SlotDesc *)(b.pool + b.off_desc);
    const void *tabs = b.pool + b.off_tabs;
    auto *act = (const int *)(b.pool + b.off_active);
    int *counter = persistent ? (int *)(b.pool + b.off_counter) : nullptr;
    const dim3 blk(b.threads), grd(grid);
#define LBM_SLOTS_T(SS, RM, MT)                                                                  \
    hipLaunchKernelGGL((k_slots<SS, RM, MT>), grd, blk, lds, b.stream, b.pool, descs, tabs, act,  \
                       nact, counter, quantum)
#define LBM_SLOTS(SS, RM)                                                                        \
    do {                                                                                         \
        if (b.threads <= 256) LBM_SLOTS_T(SS, RM, 256);                                          \
        else if (b.threads <= 512) LBM_SLOTS_T(SS, RM, 512);                                     \
        else if (b.threads <= 768) LBM_SLOTS_T(SS, RM, 768);                                     \
        else LBM_SLOTS_T(SS, RM, 1024);                                                          \
    } while (0)
    if (b.st == Storage::F32) {
        if (rmax == 1) LBM_SLOTS(Storage::F32, 1); else LBM_SLOTS(Storage::F32, 2);
    } else if (b.st == Storage::F16DEV) {
        if (rmax == 1) LBM_SLOTS(Storage::F16DEV, 1); else LBM_SLOTS(Storage::F16DEV, 2);
    } else if (b.st == Storage::F32SR) {
        if (rmax == 1) LBM_SLOTS(Storage::F32SR, 1); else LBM_SLOTS(Storage::F32SR, 2);
    } else {
        if (rmax == 1) LBM_SLOTS(Storage::F32RAW, 1); else LBM_SLOTS(Storage::F32RAW, 2);
    }
#undef LBM_SLOTS
#undef LBM_SLOTS_T
    ++b.launches;
    return hip_ok(hipGetLastError(), "batched kernel launch");
}

// Admit queued requests into free slots while pool bytes allow.
static int admit(Batch &b, bool all_or_error) {
    std::deque<Req> keep;
    while (!b.queue.empty()) {
        Req r = b.queue.front();
        b.queue.pop_front();
        size_t off = 0;
        if (b.free_slots.empty() || !b.alloc(b.state_bytes(r), off)) {
            keep.push_back(r);
            continue;
        }
        const int slot = b.free_slots.back();
        b.free_slots.pop_back();
        SlotDesc &d = b.h_desc[slot];
        std::memset(&d, 0, sizeof(d));
        d.set = r.set;
        d.ny = r.ny;
        d.check_every = r.check_every;
        d.status = kRunning;
        d.fresh = 1;
        d.tol = r.tol;
        d.max_steps = r.max_steps;
        d.mdot_scale = r.mdot_scale;
        d.pop_off = off;
        std::memcpy(d.apart, r.apart0, sizeof(d.apart));
        d.sc = r.sc;
        d.scd = r.scd;
        b.active.push_back({slot, r, off, b.state_bytes(r)});
    }
    b.queue = keep;
    if (all_or_error && !b.queue.empty())
        return fail(LBM_E_NO_MEMORY, "batch: queued requests do not all fit the slots / pool");
    return LBM_OK;
}

static int harvest(Batch &b) {
    std::vector<Batch::Act> still;
    for (auto &a : b.active) {
        const SlotDesc &d = b.h_desc[a.slot];
        if (d.status == kRunning) {
            still.push_back(a);
            continue;
        }
        lbm_result_t r{};
        r.req_id = a.req.id;
        r.status = d.status == kConverged ? LBM_OK
                   : d.status == kCapped  ? LBM_E_NOT_CONVERGED
                                          : LBM_E_DEVICE;
        r.ny = a.req.ny;
        r.steps = d.steps;
        r.mdot = d.mdot;
        r.kn = a.req.kn;
        b.done.push_back(r);
        b.release(a.off, a.bytes);
        b.free_slots.push_back(a.slot);
    }
    b.active = still;
    return LBM_OK;
}

static void take_results(Batch &b, lbm_result_t *out, int cap, int *n_out) {
    int n = 0;
    while (n < cap && !b.done.empty() && out) {
        out[n++] = b.done.front();
        b.done.erase(b.done.begin());
    }
    if (n_out) *n_out = n;
}

static int upload(Batch &b) {
    const int nact = (int)b.active.size();
    for (int k = 0; k < nact; ++k) b.h_active[k] = b.active[k].slot;
    hipError_t e = hipMemcpyAsync(b.pool + b.off_desc, b.h_desc, sizeof(SlotDesc) * b.max_slots,
                                  hipMemcpyHostToDevice, b.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.pool + b.off_active, b.h_active, sizeof(int) * std::max(1, nact),
                           hipMemcpyHostToDevice, b.stream);
    return hip_ok(e, "batch upload");
}

static int download(Batch &b) {
    hipError_t e = hipMemcpyAsync(b.h_desc, b.pool + b.off_desc, sizeof(SlotDesc) * b.max_slots,
                                  hipMemcpyDeviceToHost, b.stream);
    return hip_ok(e, "batch download");
}

static size_t launch_lds(const Batch &b, int *rmax) {
    size_t lds = 0;
    int maxny = 0;
    for (auto &a : b.active) {
        lds = std::max(lds, b.lds_bytes(a.req));
        maxny = std::max(maxny, a.req.ny);
    }
    *rmax = maxny > b.threads ? 2 : 1;
    return lds;
}

static int serve_launch(Batch &b) {
    if (b.active.empty()) return LBM_OK;
    int rc = upload(b);
    if (rc) return rc;
    int rmax = 1;
    const size_t lds = launch_lds(b, &rmax);
    rc = launch_slots(b, (int)b.active.size(), false, b.quantum, lds, rmax, (int)b.active.size());
    if (rc) return rc;
    rc = download(b);
    if (rc) return rc;
    rc = hip_ok(hipEventRecord(b.ev, b.stream), "event record");
    if (rc) return rc;
    b.inflight = true;
    return LBM_OK;
}

// Resident workgroups of a persistent launch: slots_per_cu per CU as far as
// the LDS of a CU allows, never more than the channels.
static int persistent_grid(const Batch &b, size_t lds, int nact) {
    const int per_cu = std::max<int>(1, (int)(b.max_lds / std::max<size_t>(lds, 1)));
    return std::max(1, std::min<int>(nact, b.cus * std::min(per_cu, b.slots_per_cu)));
}

// One persistent launch over all active slots. The launch (work-counter reset
// and the slot kernel, whose arguments are fixed pool addresses and the
// channel count) is captured in a HIP graph once per launch shape and
// replayed on later runs of the same shape; the slot table travels by copies
// outside the graph.
static int persistent_run(Batch &b) {
    if (b.active.empty()) return LBM_OK;
    // the device work queue hands channels out in this order
    if (b.order == LBM_BATCH_LONGEST_FIRST)   // LPT: balances the makespan
        std::stable_sort(b.active.begin(), b.active.end(),
                         [](const Batch::Act &x, const Batch::Act &y) { return x.req.est > y.req.est; });
    else
        std::stable_sort(b.active.begin(), b.active.end(),
                         [](const Batch::Act &x, const Batch::Act &y) { return x.req.seq < y.req.seq; });
    int rc = upload(b);
    if (rc) return rc;
    int rmax = 1;
    const size_t lds = launch_lds(b, &rmax);
    const int nact = (int)b.active.size();
    const int grid = persistent_grid(b, lds, nact);
    hipGraphExec_t exec = nullptr;
    for (const auto &g : b.graphs)
        if (g.nact == nact && g.grid == grid && g.threads == b.threads && g.rmax == rmax && g.lds == lds)
            exec = g.exec;
    hipError_t e = hipSuccess;
    if (exec) {
        ++b.graph_replays;
    } else {
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_ok(e, "graph capture begin");
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, b.stream,
                           (int *)(b.pool + b.off_counter));
        rc = launch_slots(b, nact, true, INT64_MAX, lds, rmax, grid);
        e = hipStreamEndCapture(b.stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_ok(e, "graph capture end");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_ok(e, "graph instantiate");
        if (b.graphs.size() >= 8) {   // the stream is idle here: runs are blocking
            (void)hipGraphExecDestroy(b.graphs.front().exec);
            b.graphs.erase(b.graphs.begin());
        }
        b.graphs.push_back({nact, grid, b.threads, rmax, lds, exec});
    }
    e = hipGraphLaunch(exec, b.stream);
    if (e == hipSuccess) rc = download(b);
    if (e == hipSuccess && !rc) e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) return hip_ok(e, "graph launch");
    if (rc) return rc;
    return harvest(b);
}

}  // namespace lbm

using namespace lbm;

extern "C" int lbm_batch_create(int max_slots, int storage, void *pool, size_t pool_bytes,
                                void *stream, lbm_batch_t **out) {
    if (!out || max_slots < 1 || !pool || (uintptr_t)pool % 256)
        return fail(LBM_E_INVALID, "lbm_batch_create: bad arguments");
    *out = nullptr;
    if (storage != LBM_F32 && storage != LBM_F16DEV && storage != LBM_F32RAW && storage != LBM_F32SR)
        return fail(LBM_E_UNSUPPORTED,
                    "lbm_batch_create: batched storage must be F32, F16DEV, F32RAW or F32SR");
    auto *b = new Batch();
    b->max_slots = max_slots;
    b->st = (Storage)storage;
    b->elem = storage == LBM_F16DEV ? 2 : 4;
    b->pool = (unsigned char *)pool;
    b->pool_bytes = pool_bytes;
    b->stream = (hipStream_t)stream;
    b->off_desc = 0;
    b->off_tabs = al(sizeof(SlotDesc) * max_slots);
    // the tables in the precision of the batch's collision
    b->off_counter = b->off_tabs + al(sizeof(PairTable<double>) * kBatchSets);
    b->off_active = b->off_counter + kAl;
    b->off_heap = b->off_active + al(sizeof(int) * max_slots);
    if (b->off_heap >= pool_bytes) {
        delete b;
        return fail(LBM_E_NO_MEMORY, "lbm_batch_create: pool too small for the slot table");
    }
    b->free_blocks[b->off_heap] = pool_bytes - b->off_heap;
    for (int s = max_slots - 1; s >= 0; --s) b->free_slots.push_back(s);
    hipError_t e = hipHostMalloc((void **)&b->h_desc, sizeof(SlotDesc) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_active, sizeof(int) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    int dev = 0, lds = 0, cus = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        if (b->h_desc) (void)hipHostFree(b->h_desc);
        if (b->h_active) (void)hipHostFree(b->h_active);
        delete b;
        return fail(LBM_E_DEVICE, std::string("lbm_batch_create: ") + hipGetErrorString(e));
    }
    std::memset(b->h_desc, 0, sizeof(SlotDesc) * max_slots);
    b->max_lds = (size_t)lds;
    b->cus = std::max(1, cus);
    *out = reinterpret_cast<lbm_batch_t *>(b);
    return LBM_OK;
}

extern "C" int lbm_batch_destroy(lbm_batch_t *h) {
    if (!h) return LBM_OK;
    Batch *b = reinterpret_cast<Batch *>(h);
    if (b->inflight) (void)hipEventSynchronize(b->ev);
    (void)hipStreamSynchronize(b->stream);
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    if (b->h_active) (void)hipHostFree(b->h_active);
    delete b;
    return LBM_OK;
}

namespace lbm {
int problem_params(const Dvm &d, const lbm_problem_t &p, lbm_params_t &par, void *tab, void *sc,
                   bool f64);
}

extern "C" int lbm_batch_submit(lbm_batch_t *h, const lbm_dvm_t *dvm, const lbm_problem_t *prob,
                                double tol, int check_every, int64_t max_steps, uint64_t req_id) {
    if (!h || !dvm || !prob || !(tol > 0) || check_every < 1 || max_steps < 0)
        return fail(LBM_E_INVALID, "lbm_batch_submit: bad arguments");
    Batch &b = *reinterpret_cast<Batch *>(h);
    const Dvm &d = *reinterpret_cast<const Dvm *>(dvm);
    if (prob->dim != 2 || prob->nx != 1)
        return fail(LBM_E_UNSUPPORTED, "lbm_batch_submit: batched solves are 2D channels with nx = 1");
    if (prob->storage != (int)b.st)
        return fail(LBM_E_INVALID, "lbm_batch_submit: storage differs from the batch's");
    if (prob->accommodation != 1.0)
        return fail(LBM_E_UNSUPPORTED, "lbm_batch_submit: the batched kernel has fully diffuse walls");
    if (prob->hermite_order > 4)
        return fail(LBM_E_UNSUPPORTED, "lbm_batch_submit: the batched kernel implements Hermite orders up to 4");
    const int set = match_set(d);
    if (set != SetD2V17::ID && set != SetD2V37::ID)
        return fail(LBM_E_UNSUPPORTED, "lbm_batch_submit: the batched kernel handles D2V17 and D2V37");
    Req r{};
    lbm_params_t par;
    PairTable<float> tab;
    PairTable<double> tabd;
    int rc = problem_params(d, *prob, par, &tab, &r.sc, false);
    if (rc == LBM_OK && b.st == Storage::F32SR) rc = problem_params(d, *prob, par, &tabd, &r.scd, true);
    if (rc) return rc;
    if (r.sc.halo > 4) return fail(LBM_E_UNSUPPORTED, "lbm_batch_submit: wall halo above 4");
    if (b.tab_set[set]) {
        for (int q = 0; q < kMaxPairs; ++q)
            if (b.tabs[set].w[q] != tab.w[q])
                return fail(LBM_E_UNSUPPORTED, "lbm_batch_submit: a second weight table for one velocity set");
    } else {
        b.tabs[set] = tab;
        b.tab_set[set] = true;
        hipError_t e =
            b.st == Storage::F32SR
                ? hipMemcpy(b.pool + b.off_tabs + sizeof(PairTable<double>) * set, &tabd,
                            sizeof(tabd), hipMemcpyHostToDevice)
                : hipMemcpy(b.pool + b.off_tabs + sizeof(PairTable<float>) * set, &tab,
                            sizeof(tab), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_ok(e, "lbm_batch_submit: table upload");
    }
    r.id = req_id;
    r.set = set;
    r.ny = prob->ny;
    r.kn = prob->kn;
    r.tol = tol;
    r.check_every = check_every;
    r.max_steps = max_steps;
    r.mdot_scale = par.mdot_scale;
    // work ~ nodes x steps to converge, steps ~ c ny / tau (a diffusion time)
    r.est = (double)prob->ny * prob->ny * d.c / par.tau;
    r.seq = b.next_seq++;
    // rest-state wall partials: w rho0 of the populations leaving from each wall row
    for (int f = 0; f < 2; ++f)
        for (int rr = 0; rr < 4; ++rr) {
            double a = 0.0;
            for (int v = 0; v < d.V; ++v) {
                const int ey = d.vel[3 * v + 1];
                if ((f == 0 && ey < -rr) || (f == 1 && ey > rr)) a += d.w[v] * prob->rho0;
            }
            r.apart0[f][rr] = a;
        }
    if (b.lds_bytes(r) > b.max_lds || (size_t)prob->ny > 2u * 1024u)
        return fail(LBM_E_NO_MEMORY, "lbm_batch_submit: channel does not fit one workgroup's LDS");
    // a thread steps at most two rows: refuse here rather than after admission
    if (prob->ny > 2 * b.threads)
        return fail(LBM_E_INVALID, "lbm_batch_submit: ny above twice the workgroup size");
    if (b.state_bytes(r) > b.pool_bytes - b.off_heap)
        return fail(LBM_E_NO_MEMORY, "lbm_batch_submit: channel larger than the pool");
    b.queue.push_back(r);
    return LBM_OK;
}

extern "C" int lbm_batch_poll(lbm_batch_t *h, lbm_result_t *out, int cap, int *n_out) {
    if (!h) return fail(LBM_E_INVALID, "lbm_batch_poll: null handle");
    Batch &b = *reinterpret_cast<Batch *>(h);
    if (b.inflight) {
        const hipError_t e = hipEventQuery(b.ev);
        if (e == hipSuccess) {
            b.inflight = false;
            int rc = harvest(b);
            if (rc) return rc;
        } else if (e != hipErrorNotReady) {
            return hip_ok(e, "lbm_batch_poll");
        }
    }
    if (!b.inflight) {
        int rc = admit(b, false);
        if (rc) return rc;
        for (auto &a : b.active)
            if (a.req.ny > 2 * b.threads)
                return fail(LBM_E_INVALID, "lbm_batch_poll: workgroup too small for a resident channel");
        rc = serve_launch(b);
        if (rc) return rc;
    }
    take_results(b, out, cap, n_out);
    return LBM_OK;
}

extern "C" int lbm_batch_drain(lbm_batch_t *h, lbm_result_t *out, int cap, int *n_out) {
    if (!h) return fail(LBM_E_INVALID, "lbm_batch_drain: null handle");
    Batch &b = *reinterpret_cast<Batch *>(h);
    int total = 0;
    for (;;) {
        if (b.inflight) {
            hipError_t e = hipEventSynchronize(b.ev);
            if (e != hipSuccess) return hip_ok(e, "lbm_batch_drain");
        }
        int n = 0;
        int rc = lbm_batch_poll(h, out ? out + total : nullptr, out ? cap - total : 0, &n);
        if (rc) return rc;
        total += n;
        if (!b.inflight && b.active.empty() && b.queue.empty()) break;
    }
    if (n_out) *n_out = total;
    return LBM_OK;
}

extern "C" int lbm_batch_run_persistent(lbm_batch_t *h, lbm_result_t *out, int cap, int *n_out) {
    if (!h) return fail(LBM_E_INVALID, "lbm_batch_run_persistent: null handle");
    Batch &b = *reinterpret_cast<Batch *>(h);
    if (b.inflight) {
        hipError_t e = hipEventSynchronize(b.ev);
        if (e != hipSuccess) return hip_ok(e, "lbm_batch_run_persistent");
        b.inflight = false;
        harvest(b);
    }
    int rc = admit(b, true);
    if (rc) return rc;
    for (auto &a : b.active)
        if (a.req.ny > 2 * b.threads)
            return fail(LBM_E_INVALID, "lbm_batch_run_persistent: workgroup too small for a channel");
    rc = persistent_run(b);
    if (rc) return rc;
    take_results(b, out, cap, n_out);
    return LBM_OK;
}

extern "C" int lbm_batch_tune(lbm_batch_t *h, int threads, int quantum, int slots_per_cu,
                              int order) {
    if (!h || threads < 64 || threads > 1024 || threads % 64 || quantum < 1 || slots_per_cu < 0 ||
        slots_per_cu > 16 || order < 0 || order > LBM_BATCH_SUBMIT_ORDER)
        return fail(LBM_E_INVALID, "lbm_batch_tune: bad arguments");
    Batch &b = *reinterpret_cast<Batch *>(h);
    int maxny = 0;
    for (auto &r : b.queue) maxny = std::max(maxny, r.ny);
    for (auto &a : b.active) maxny = std::max(maxny, a.req.ny);
    if (2 * threads < maxny)
        return fail(LBM_E_INVALID, "lbm_batch_tune: a queued or resident channel has more than "
                                   "twice that many rows");
    b.threads = threads;
    b.quantum = quantum;
    if (slots_per_cu > 0) b.slots_per_cu = slots_per_cu;
    if (order > 0) b.order = order;
    return LBM_OK;
}

// Autotuner of the persistent launch: every workgroup size that can hold the
// tallest channel (which fixes the rows per thread: one, or two where the
// channel is taller than the workgroup) times 1 to 4 resident workgroups per
// CU times both work-queue orders, each timed on a trial of the queued
// requests capped at trial_steps steps. Results do not depend on the choice.
extern "C" int lbm_batch_autotune(lbm_batch_t *h, int trial_steps, lbm_batch_tuning_t *out) {
    if (!h || trial_steps < 1) return fail(LBM_E_INVALID, "lbm_batch_autotune: bad arguments");
    Batch &b = *reinterpret_cast<Batch *>(h);
    if (b.inflight || !b.active.empty())
        return fail(LBM_E_INVALID, "lbm_batch_autotune: batch must be idle");
    lbm_batch_tuning_t res{b.threads, b.slots_per_cu, b.order, 0, 0.0f};
    if (b.queue.empty()) {
        if (out) *out = res;
        return LBM_OK;
    }
    const std::deque<Req> saved = b.queue;
    int maxny = 0;
    size_t maxlds = 0;
    for (auto &r : saved) {
        maxny = std::max(maxny, r.ny);
        maxlds = std::max(maxlds, b.lds_bytes(r));
    }
    const int lds_per_cu = std::max<int>(1, (int)(b.max_lds / std::max<size_t>(maxlds, 1)));
    const int cands[] = {256, 384, 512, 768, 1024};
    float best = 1e30f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(LBM_E_DEVICE, "lbm_batch_autotune: events");
    int rc = LBM_OK;
    for (int th : cands) {
        if (2 * th < maxny) continue;
        for (int sp = 1; sp <= std::min(4, lds_per_cu) && rc == LBM_OK; ++sp) {
            // more resident workgroups than 2048 threads per CU gain nothing
            if (sp > 1 && sp * th > 2048) continue;
            for (int order = LBM_BATCH_LONGEST_FIRST; order <= LBM_BATCH_SUBMIT_ORDER; ++order) {
                b.threads = th;
                b.slots_per_cu = sp;
                b.order = order;
                b.queue = saved;
                for (auto &r : b.queue) r.max_steps = std::min<int64_t>(r.max_steps, trial_steps);
                rc = admit(b, true);
                if (rc) break;
                (void)hipEventRecord(e0, b.stream);
                rc = persistent_run(b);   // harvests every trial channel
                (void)hipEventRecord(e1, b.stream);
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                b.done.clear();
                if (rc) break;
                ++res.trials;
                if (ms < best) {
                    best = ms;
                    res.threads = th;
                    res.slots_per_cu = sp;
                    res.order = order;
                    res.trial_ms = ms;
                }
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b.queue = saved;
    b.threads = res.threads;
    b.slots_per_cu = res.slots_per_cu;
    b.order = res.order;
    if (out) *out = res;
    return rc;
}

extern "C" int lbm_batch_stats(const lbm_batch_t *h, lbm_batch_stats_t *out) {
    if (!h || !out) return fail(LBM_E_INVALID, "lbm_batch_stats: null argument");
    const Batch &b = *reinterpret_cast<const Batch *>(h);
    out->active = (int)b.active.size();
    out->queued = (int)b.queue.size();
    out->done = (int)b.done.size();
    out->threads = b.threads;
    out->quantum = b.quantum;
    out->slots_per_cu = b.slots_per_cu;
    out->order = b.order;
    out->graph_replays = b.graph_replays;
    out->launches = b.launches;
    out->pool_used = b.used;
    out->pool_free = b.heap_free();
    return LBM_OK;
}
