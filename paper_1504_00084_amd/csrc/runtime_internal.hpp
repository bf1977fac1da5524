// Internals of the host runtime shared by its source files (runtime.cpp:
// contexts, instances, requests, scheduler; mesh_step.cpp: the mesh step
// around the interface estimate).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "mesh_sdd.h"
#include "msdd_device.hpp"
#include "msdd_kernels.hpp"

namespace msdd_rt {

// Sets the calling thread's last-error text (mesh_sdd_last_error) and
// returns `code`.
int fail(int code, const char *fmt, ...);

// Status of an exception caught at the C-ABI (called inside a catch block):
// E_NOMEM for a failed host allocation (std::bad_alloc) or any other
// exhausted host resource (e.g. a thread that cannot be started).  No
// exception crosses the ABI.
int abi_exception() noexcept;

#define HIP_TRY(expr)                                                                                     \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail(MESH_SDD_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

using Clock = std::chrono::steady_clock;

inline double ms_since(Clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Free device blocks kept for reuse, keyed by their exact size (requests of
// the same shape reuse the same blocks, so steady-state solves call neither
// hipMalloc nor hipFree).  Bounded: blocks beyond `cap` bytes are freed.
struct DevPool {
    std::mutex mu;
    std::multimap<size_t, void *> free_blocks;
    size_t pooled = 0;
    size_t cap = (size_t)1 << 30;
    ~DevPool() { trim(0); }
    void *get(size_t n)
    {
        {
            std::lock_guard<std::mutex> g(mu);
            auto it = free_blocks.find(n);
            if (it != free_blocks.end()) {
                void *p = it->second;
                free_blocks.erase(it);
                pooled -= n;
                return p;
            }
        }
        void *p = nullptr;
        if (hipMalloc(&p, n) != hipSuccess) {
            trim(0);   // give cached blocks back and try once more
            if (hipMalloc(&p, n) != hipSuccess) return nullptr;
        }
        return p;
    }
    void put(void *p, size_t n) noexcept   // called from destructors: never throws
    {
        std::lock_guard<std::mutex> g(mu);
        try {
            free_blocks.emplace(n, p);
        } catch (...) {   // no host memory for the pool's bookkeeping: free the block
            (void)hipFree(p);
            return;
        }
        pooled += n;
        while (pooled > cap && !free_blocks.empty()) {
            auto it = free_blocks.begin();
            pooled -= it->first;
            (void)hipFree(it->second);
            free_blocks.erase(it);
        }
    }
    void trim(size_t keep)
    {
        std::lock_guard<std::mutex> g(mu);
        while (pooled > keep && !free_blocks.empty()) {
            auto it = free_blocks.begin();
            pooled -= it->first;
            (void)hipFree(it->second);
            free_blocks.erase(it);
        }
    }
};

// A fixed region of device memory handed out front to back in 256-byte
// aligned pieces (the no-allocation solve carves its buffers from the
// library's static scratch array this way).  Nothing is ever freed.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    size_t used = 0;
    void *take(size_t n)
    {
        n = n == 0 ? 256 : (n + 255) / 256 * 256;
        if (!base || used + n > size) return nullptr;
        void *p = base + used;
        used += n;
        return p;
    }
};

// Device allocation owned by one object (from a pool when one is given), or
// a piece of an Arena that it only borrows (never freed by it).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevPool *pool = nullptr;
    Arena *arena = nullptr;   // set: alloc takes from the arena, release frees nothing
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p && !arena) {
            if (pool)
                pool->put(p, bytes);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t n)
    {
        release();
        n = n == 0 ? 256 : (n + 255) / 256 * 256;
        if (arena) {
            p = arena->take(n);
            if (!p) return hipErrorOutOfMemory;
            bytes = n;
            return hipSuccess;
        }
        if (pool) {
            p = pool->get(n);
            if (!p) return hipErrorOutOfMemory;
            bytes = n;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess)
            bytes = n;
        else
            p = nullptr;
        return e;
    }
    // grow-only reuse
    hipError_t reserve(size_t n)
    {
        if (n <= bytes && p) return hipSuccess;
        return alloc(n);
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// The two timing events of a launch, destroyed on every way out of the scope.
struct TimerEvents {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TimerEvents() = default;
    TimerEvents(const TimerEvents &) = delete;
    TimerEvents &operator=(const TimerEvents &) = delete;
    hipError_t create()
    {
        hipError_t e = hipEventCreate(&e0);
        if (e != hipSuccess) {
            e0 = nullptr;
            return e;
        }
        e = hipEventCreate(&e1);
        if (e != hipSuccess) e1 = nullptr;
        return e;
    }
    ~TimerEvents()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace msdd_rt

using msdd_rt::Clock;
using msdd_rt::DevBuf;
using msdd_rt::DevPool;
using msdd::InstView;

// ---------------------------------------------------------------------------
// Objects behind the opaque handles
// ---------------------------------------------------------------------------
struct Request;

// The interface nodes that run paths under one sampling stride (1: all of
// them): device lists node_i[Ms], node_j[Ms], node_r[Ms] (int32, in that
// order, contiguous) in rank order.
// A run of consecutive positions of a node list whose nodes lie in one
// block of the grid, and the window of node tables the windowed kernel
// stages in LDS for them (nodes [i0, i0 + tw) x [j0, j0 + th)).
struct BlockRun {
    int32_t pos_begin, pos_end;
    int32_t i0, j0, tw, th;
    int32_t kind;   // 0: (rho, dt rho_xi) per node; 1: also dt rho_eta per node
};

// The nodes that run paths for one interface stride.  They are stored in
// block order (grid blocks of the windowed kernel, ranks ascending inside a
// block), so that a request's items -- node-major over these positions --
// visit the grid block by block; the rank of each position is its random
// stream and result slot, so the order does not change any result.
struct SampleSet {
    int stride = 1;
    int kind = 0, margin = 0;            // block layout: window kind and margin (see BlockRun)
    int32_t Ms = 0;
    DevBuf lists;
    std::vector<BlockRun> blocks;        // covers positions [0, Ms) in order
    std::vector<int32_t> pos_of_rank;    // position of interface rank r, or -1 (not sampled)
    const int32_t *node_i() const { return lists.as<int32_t>(); }
    const int32_t *node_j() const { return lists.as<int32_t>() + Ms; }
    const uint32_t *node_r() const { return reinterpret_cast<const uint32_t *>(lists.as<int32_t>() + 2 * (size_t)Ms); }
};

struct mesh_sdd {
    mesh_sdd_ctx *ctx = nullptr;
    mesh_sdd_desc d{};
    int32_t M = 0;
    std::vector<int32_t> node_i, node_j;
    // sample sets by (stride, window kind, window margin): the stride-1 set
    // of the default layout is built at create, the others on first use
    // (under ctx->gpu_mu), and all live until destroy -- a staged request
    // keeps a pointer to its set, so a set is never rebuilt in place
    std::map<std::tuple<int, int, int>, std::unique_ptr<SampleSet>> samples;
    DevBuf rho_in, rho, rho_xi, rho_eta;    // FP64 monitor staging and node tables
    DevBuf rho_f, rhox_f, rhoy_f;           // FP32 node tables of rho, dt rho_xi, dt rho_eta (staged in LDS
                                            // whole or in windows)
    DevBuf cells;                           // FP32 cell data: the dt rho_eta corners alone (one float4 per
                                            // cell), then the 48-B records (rho and dt rho_xi corners, the
                                            // dt rho_eta corners again); one allocation, below 2^32 bytes
    DevBuf node_rank;                       // [n_eta][n_xi] interface rank or -1
    DevBuf node_ij;                         // interface nodes in rank order: i[M], then j[M]
    bool monitor_set = false;
    std::atomic<int> inflight{0};
    size_t resident_bytes = 0;
};

struct Request {
    uint64_t ticket = 0;
    mesh_sdd *inst = nullptr;      // valid until the request finishes
    int32_t M = 0;                 // interface nodes (kept for poll after finish)
    int32_t Ms = 0;                // of which run paths (all unless subsampled)
    int stride = 1;                // interface sampling stride
    const SampleSet *ss = nullptr; // set by stage_request
    int64_t N = 0;
    uint32_t mesh_step = 0;
    int chunk_paths = 0;
    // host snapshots of host inputs
    std::vector<double> hx, hy, hb0, hb1;
    // device buffers owned by the request
    DevBuf x64, y64, b0, b1, xpad, ypad, xpad_f, ypad_f, b0f, b1f;
    DevBuf view, partials, spans, out, steps_total;
    InstView v{};
    size_t n_items = 0;            // FP32 work items (node-major, see WorkRange)
    size_t next_item = 0;          // first item not yet handed to a tick
    size_t done_items = 0;
    uint32_t chunks_per_node = 0;
    size_t cost_bytes = 0;
    // completion
    int status = MESH_SDD_PENDING;
    std::string error;
    std::vector<double> host_out;  // 5 * M
    uint64_t executed_steps = 0;
    double device_ms = 0.0;
    Clock::time_point t_submit, t_done;
    bool finished = false;
    bool admitted = false;
    bool cancelled = false;
};

// Holds one in-flight count on each instance added, for the duration of a
// blocking call: released when the hold goes out of scope, also when the call
// leaves by an exception (the count never leaks, so destroy never blocks).
struct InflightHold {
    std::vector<mesh_sdd *> held;
    void add(mesh_sdd *i)
    {
        held.push_back(i);   // may throw: then nothing was counted
        i->inflight.fetch_add(1);
    }
    ~InflightHold()
    {
        for (mesh_sdd *i : held) i->inflight.fetch_sub(1);
    }
};

struct TuneKey {
    int n_xi, n_eta, per_xi, per_eta;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(n_xi, n_eta, per_xi, per_eta) < std::tie(o.n_xi, o.n_eta, o.per_xi, o.per_eta);
    }
};

struct mesh_sdd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cu_count = 0;
    size_t budget = 0;

    DevPool pool;        // recycled request buffers (declared before users)
    std::mutex gpu_mu;   // serialises use of the stream and the launch scratch below
    DevBuf head, views, ranges;
    DevBuf jobs;         // job list of windowed launches (grow-only)
    DevBuf ends;         // item end states of the LDS table and window launches (grow-only)

    std::mutex mu;       // guards everything below
    std::condition_variable cv, done_cv;
    size_t in_use = 0;
    int n_instances = 0;
    std::deque<std::shared_ptr<Request>> queue;    // submitted, not admitted
    std::vector<std::shared_ptr<Request>> running; // admitted, not finished
    std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    // stats
    uint64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, ticks = 0, executed = 0;
    double busy_ms = 0.0;
    std::vector<double> latencies;

    // launch shapes: a fixed override, the tuned shape per bucket (launches of
    // one instance, and the per-instance knobs everywhere), and the tuned
    // launch-wide knobs of multi-instance launches
    bool has_override = false;
    mesh_sdd_launch override_launch{};
    std::map<TuneKey, mesh_sdd_launch> tuned;
    bool has_batch_tuned = false;
    mesh_sdd_launch batch_tuned{};
};

namespace msdd_rt {
int install_monitor(mesh_sdd *inst, hipStream_t st);

// The static device scratch of the no-allocation solve (noalloc.hip): its
// size, the one-time lookup of its address on a device (the caller has made
// that device current), and that address with the lock its users hold.
size_t scratch_capacity();
hipError_t scratch_resolve(int device);
int scratch_region(int device, void **base, std::mutex **use);

// Ranks of the interface nodes that run paths under `stride` (0 or 1: all),
// in rank order.  The stride must have passed the step validation.
std::vector<int32_t> sampled_ranks(const mesh_sdd &inst, int stride);
}  // namespace msdd_rt
