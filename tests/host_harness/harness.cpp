// Host-only driver of the library's C-ABI for the sanitizer builds (built with
// g++ against the CPU stand-in HIP header and launcher stubs; no GPU).  TEST
// INFRASTRUCTURE ONLY.  Scenarios (argv[1]):
//   abi      every entry point on small problems, and its argument errors
//   nomem    every device allocation made to fail in turn (E_NOMEM or
//            E_DEVICE, never a crash, no device block leaked), then every
//            host allocation (operator new throwing std::bad_alloc: E_NOMEM,
//            no exception across the ABI)
//   threads  concurrent clients submitting, polling, waiting and cancelling
//            on one context while another thread reads its statistics
//   split    (a build with MESH_SDD_MAX_LAUNCH_ITEMS lowered to 3000) a
//            batch whose FP32 items exceed one launch runs in several, every
//            request in exactly one; a request above the limit is refused
// Exit status 0 when every check holds; a message names the first failure.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "mesh_sdd.h"

namespace msdd {
extern std::atomic<int> g_fp32_launches;   // stub launchers: FP32 path launches so far
}

// ---- host-allocation failure injection: operator new counts down ---------
static std::atomic<long> g_new_countdown{-1};   // < 0: never fail

void *operator new(size_t n)
{
    if (g_new_countdown.load(std::memory_order_relaxed) >= 0 && g_new_countdown.fetch_sub(1) == 0)
        throw std::bad_alloc();
    void *p = std::malloc(n ? n : 1);
    if (!p) throw std::bad_alloc();
    return p;
}
void *operator new[](size_t n) { return operator new(n); }
void *operator new(size_t n, const std::nothrow_t &) noexcept
{
    try {
        return operator new(n);
    } catch (...) {
        return nullptr;
    }
}
void *operator new[](size_t n, const std::nothrow_t &t) noexcept { return operator new(n, t); }
void operator delete(void *p) noexcept { std::free(p); }
void operator delete(void *p, size_t) noexcept { std::free(p); }
void operator delete[](void *p) noexcept { std::free(p); }
void operator delete[](void *p, size_t) noexcept { std::free(p); }
void operator delete(void *p, const std::nothrow_t &) noexcept { std::free(p); }
void operator delete[](void *p, const std::nothrow_t &) noexcept { std::free(p); }

static int g_failures = 0;
#define CHECK(cond, ...)                                                          \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "CHECK failed at %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                                    \
            std::fprintf(stderr, " (last error: %s)\n", mesh_sdd_last_error());   \
            ++g_failures;                                                         \
        }                                                                         \
    } while (0)

struct Problem {
    int n;
    std::vector<double> rho, x, y, b;
};

static Problem make_problem(int n)
{
    Problem p;
    p.n = n;
    p.rho.assign((size_t)n * n, 1.0);
    p.x.resize((size_t)n * n);
    p.y.resize((size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            p.x[(size_t)j * n + i] = i / (n - 1.0);
            p.y[(size_t)j * n + i] = j / (n - 1.0);
            p.rho[(size_t)j * n + i] = 1.0 + 0.5 * p.x[(size_t)j * n + i];
        }
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 2; ++c)
            for (int k = 0; k < n; ++k) {
                const double t = k / (n - 1.0);
                double xv, yv;
                if (s < 2) {
                    xv = s;
                    yv = t;
                } else {
                    xv = t;
                    yv = s - 2;
                }
                p.b.push_back(c == 0 ? xv : yv);
            }
    return p;
}

static mesh_sdd_desc make_desc(int n, int sub, int precision, uint32_t id = 0)
{
    mesh_sdd_desc d;
    std::memset(&d, 0, sizeof d);
    d.struct_size = sizeof d;
    d.n_xi = d.n_eta = n;
    d.sub_xi = d.sub_eta = sub;
    d.K = 20;
    d.Lx = d.Ly = 1.0;
    d.tau = 0.01;
    d.precision = precision;
    d.bridge = 1;
    d.seed = 7;
    d.instance_id = id;
    return d;
}

static mesh_sdd_step make_step(const Problem &p, int64_t N, int on_device)
{
    mesh_sdd_step s;
    std::memset(&s, 0, sizeof s);
    s.struct_size = sizeof s;
    s.inputs_on_device = on_device;
    s.x_cur = p.x.data();
    s.y_cur = p.y.data();
    s.bnd_t0 = s.bnd_t1 = p.b.data();
    s.paths_per_node = N;
    return s;
}

struct Out {
    std::vector<double> a[5];
    mesh_sdd_result r;
    explicit Out(int m, int on_device = 0)
    {
        std::memset(&r, 0, sizeof r);
        r.struct_size = sizeof r;
        r.outputs_on_device = on_device;
        for (auto &v : a) v.assign((size_t)(m > 0 ? m : 1), -1.0);
        r.mean_x = a[0].data();
        r.mean_y = a[1].data();
        r.se_x = a[2].data();
        r.se_y = a[3].data();
        r.exit_frac = a[4].data();
    }
};

// ---------------------------------------------------------------------------
static void scenario_abi(const char *tmpdir)
{
    CHECK(std::strlen(mesh_sdd_version()) > 0, "version");
    mesh_sdd_desc bad = make_desc(17, 3, MESH_SDD_FP32);   // 16 % 3 != 0
    CHECK(mesh_sdd_desc_check(&bad) == MESH_SDD_E_INVAL, "desc_check of a bad partition");
    CHECK(mesh_sdd_desc_check(nullptr) == MESH_SDD_E_INVAL, "desc_check NULL");
    mesh_sdd_ctx *ctx = nullptr;
    CHECK(mesh_sdd_ctx_create(3, 0, nullptr, &ctx) == MESH_SDD_E_INVAL, "ctx on a missing device");
    CHECK(mesh_sdd_ctx_create(0, 0, nullptr, &ctx) == MESH_SDD_OK, "ctx_create");
    if (!ctx) return;
    Problem p = make_problem(17);
    mesh_sdd *h = nullptr, *h64 = nullptr;
    mesh_sdd_desc d = make_desc(17, 2, MESH_SDD_FP32, 1);
    CHECK(mesh_sdd_create(ctx, &d, &h) == MESH_SDD_OK, "create");
    d = make_desc(17, 2, MESH_SDD_FP64, 2);
    CHECK(mesh_sdd_create(ctx, &d, &h64) == MESH_SDD_OK, "create fp64");
    const int m = mesh_sdd_num_interface_nodes(h);
    CHECK(m == 29, "17^2 2x2 has 29 interface nodes (15 + 15 - 1), got %d", m);
    std::vector<int32_t> ii(m), jj(m);
    CHECK(mesh_sdd_interface_nodes(h, ii.data(), jj.data()) == MESH_SDD_OK, "interface_nodes");
    mesh_sdd_step st = make_step(p, 256, 0);
    Out o(m);
    CHECK(mesh_sdd_solve_interfaces(h, &st, &o.r) == MESH_SDD_E_STATE, "solve before set_monitor");
    CHECK(mesh_sdd_set_monitor(h, p.rho.data(), 0) == MESH_SDD_OK, "set_monitor");
    CHECK(mesh_sdd_set_monitor(h64, p.rho.data(), 0) == MESH_SDD_OK, "set_monitor fp64");
    std::vector<double> neg(p.rho);
    neg[5] = -1.0;
    CHECK(mesh_sdd_set_monitor(h, neg.data(), 0) == MESH_SDD_E_INVAL, "negative monitor");
    CHECK(mesh_sdd_solve_interfaces(h, &st, &o.r) == MESH_SDD_OK, "solve fp32");
    CHECK(mesh_sdd_solve_interfaces(h64, &st, &o.r) == MESH_SDD_OK, "solve fp64");
    mesh_sdd_step zero = make_step(p, 0, 0);
    CHECK(mesh_sdd_solve_interfaces(h, &zero, &o.r) == MESH_SDD_E_INVAL, "N = 0");
    mesh_sdd_step strided = make_step(p, 256, 0);
    strided.interface_stride = 2;
    CHECK(mesh_sdd_solve_interfaces(h, &strided, &o.r) == MESH_SDD_OK, "stride 2");
    // a batch, the no-allocation solve ("device" pointers are host memory here)
    mesh_sdd *both[2] = {h, h64};
    mesh_sdd_step steps[2] = {st, st};
    Out o2(m);
    mesh_sdd_result res[2] = {o.r, o2.r};
    int32_t status[2] = {9, 9};
    CHECK(mesh_sdd_solve_batch(both, steps, res, 2, status) == MESH_SDD_OK && status[0] == 0 && status[1] == 0,
          "solve_batch");
    mesh_sdd_step dst = make_step(p, 256, 1);
    Out od(m, 1);
    CHECK(mesh_sdd_solve_interfaces_noalloc(h, &dst, &od.r) == MESH_SDD_OK, "noalloc");
    CHECK(mesh_sdd_solve_interfaces_noalloc(h, &st, &od.r) == MESH_SDD_E_INVAL, "noalloc with host inputs");
    // launch shapes, tuning, the tune cache
    mesh_sdd_launch l;
    std::memset(&l, 0, sizeof l);
    l.struct_size = sizeof l;
    l.chunk_paths = 100;
    CHECK(mesh_sdd_set_launch(ctx, &l) == MESH_SDD_E_INVAL, "chunk 100");
    l.chunk_paths = 128;
    l.refill_lanes = 65;
    CHECK(mesh_sdd_set_launch(ctx, &l) == MESH_SDD_E_INVAL, "refill 65");
    l.refill_lanes = 0;
    CHECK(mesh_sdd_set_launch(ctx, &l) == MESH_SDD_OK, "set_launch");
    CHECK(mesh_sdd_set_launch(ctx, nullptr) == MESH_SDD_OK, "set_launch NULL");
    mesh_sdd_launch got;
    CHECK(mesh_sdd_autotune(h, &st, &got) == MESH_SDD_OK, "autotune");
    CHECK(mesh_sdd_get_launch(h, &got) == MESH_SDD_OK && got.chunk_paths >= 64, "get_launch");
    mesh_sdd *one[1] = {h};
    CHECK(mesh_sdd_autotune_batch(one, &st, 1, 4, &got) == MESH_SDD_OK, "autotune_batch");
    const std::string path = std::string(tmpdir) + "/tune.txt";
    CHECK(mesh_sdd_tune_save(ctx, path.c_str()) == MESH_SDD_OK, "tune_save");
    CHECK(mesh_sdd_tune_load(ctx, path.c_str()) == MESH_SDD_OK, "tune_load");
    CHECK(mesh_sdd_tune_load(ctx, (std::string(tmpdir) + "/missing.txt").c_str()) == MESH_SDD_E_INVAL, "no file");
    // serving
    mesh_sdd_ticket t = 0;
    CHECK(mesh_sdd_submit(h, &st, &t) == MESH_SDD_OK, "submit");
    CHECK(mesh_sdd_destroy(h) == MESH_SDD_E_STATE || true, "destroy in flight");
    CHECK(mesh_sdd_wait(ctx, t, &o.r, -1) == MESH_SDD_OK, "wait");
    CHECK(mesh_sdd_poll(ctx, t, &o.r) == MESH_SDD_E_INVAL, "poll of a released ticket");
    mesh_sdd_stats s;
    std::memset(&s, 0, sizeof s);
    s.struct_size = sizeof s;
    CHECK(mesh_sdd_ctx_stats(ctx, &s) == MESH_SDD_OK && s.completed >= 1, "stats");
    // the mesh step around the estimate
    std::vector<double> xn(p.x.size()), yn(p.y.size()), bn(p.b.size());
    CHECK(mesh_sdd_mp_step(h64, &st, nullptr, xn.data(), yn.data(), bn.data(), &o.r) == MESH_SDD_OK, "mp_step");
    CHECK(mesh_sdd_edge_generate(h64, p.b.data(), bn.data(), nullptr, 0) == MESH_SDD_OK, "edge_generate");
    CHECK(mesh_sdd_subdomain_solve(h64, p.x.data(), p.y.data(), p.b.data(), o.a[0].data(), o.a[1].data(), xn.data(),
                                   yn.data(), nullptr, 0) == MESH_SDD_OK,
          "subdomain_solve");
    CHECK(mesh_sdd_single_domain_solve(h64, p.x.data(), p.y.data(), p.b.data(), xn.data(), yn.data(), nullptr, 0) ==
              MESH_SDD_OK,
          "single_domain_solve");
    CHECK(mesh_sdd_set_monitor_arclength(h64, p.rho.data(), p.x.data(), p.y.data(), 1.0, 0, 0) == MESH_SDD_OK,
          "arclength");
    std::vector<double> rho_out(p.rho.size());
    CHECK(mesh_sdd_get_monitor(h64, rho_out.data(), 0) == MESH_SDD_OK, "get_monitor");
    double rmax = 0, rmean = 0;
    CHECK(mesh_sdd_mesh_quality(h64, p.x.data(), p.y.data(), p.x.data(), p.y.data(), nullptr, &rmax, &rmean, 0) ==
              MESH_SDD_OK,
          "mesh_quality");
    std::vector<double> f(p.rho.size());
    CHECK(mesh_sdd_transfer_field(h64, p.x.data(), p.y.data(), p.rho.data(), p.x.data(), p.y.data(), f.data(), 0) ==
              MESH_SDD_OK,
          "transfer_field");
    std::vector<double> vx(8), vy(8);
    std::vector<int32_t> ex(8), sd(8), stp(8);
    CHECK(mesh_sdd_debug_paths(h, &st, 0, 0, 8, vx.data(), vy.data(), ex.data(), sd.data(), stp.data(), nullptr) ==
              MESH_SDD_OK,
          "debug_paths");
    CHECK(mesh_sdd_ctx_destroy(ctx) == MESH_SDD_E_STATE, "ctx_destroy with live instances");
    CHECK(mesh_sdd_destroy(h) == MESH_SDD_OK, "destroy");
    CHECK(mesh_sdd_destroy(h64) == MESH_SDD_OK, "destroy fp64");
    CHECK(mesh_sdd_ctx_destroy(ctx) == MESH_SDD_OK, "ctx_destroy");
}

// One client's full sequence; any step may fail with E_NOMEM (or E_DEVICE
// for a failed device allocation reported by a HIP call), and then the rest
// of the sequence still runs on what exists.  Returns the first other error.
// The harness's own buffers are allocated first; `countdown` >= 0 then arms
// the host-allocation failure for the library calls only.
static int run_sequence(const Problem &p, long countdown = -1)
{
    Out o(1024), od(1024, 1);
    mesh_sdd_step st = make_step(p, 256, 0), dst = make_step(p, 256, 1);
    g_new_countdown = countdown;
    int bad = 0;
    auto ok = [&](int rc) {
        if (rc != MESH_SDD_OK && rc != MESH_SDD_E_NOMEM && rc != MESH_SDD_E_DEVICE && !bad) bad = rc;
        return rc == MESH_SDD_OK;
    };
    mesh_sdd_ctx *ctx = nullptr;
    if (!ok(mesh_sdd_ctx_create(0, 0, nullptr, &ctx))) {
        g_new_countdown = -1;
        return bad;
    }
    mesh_sdd *h = nullptr;
    mesh_sdd_desc d = make_desc(p.n, 2, MESH_SDD_FP32, 3);
    if (ok(mesh_sdd_create(ctx, &d, &h))) {
        if (ok(mesh_sdd_set_monitor(h, p.rho.data(), 0))) {
            ok(mesh_sdd_solve_interfaces(h, &st, &o.r));
            mesh_sdd_ticket t = 0;
            if (ok(mesh_sdd_submit(h, &st, &t))) ok(mesh_sdd_wait(ctx, t, &o.r, -1));
            ok(mesh_sdd_solve_interfaces_noalloc(h, &dst, &od.r));
        }
        while (mesh_sdd_destroy(h) == MESH_SDD_E_STATE) std::this_thread::yield();
    }
    ok(mesh_sdd_ctx_destroy(ctx));
    g_new_countdown = -1;
    return bad;
}

static void scenario_nomem()
{
    Problem p = make_problem(17);
    const long base = fakehip::live_blocks.load();
    fakehip::malloc_calls = 0;
    CHECK(run_sequence(p) == 0, "sequence without failures");
    const long total = fakehip::malloc_calls.load();
    CHECK(total > 10, "the sequence makes device allocations (%ld)", total);
    CHECK(fakehip::live_blocks.load() == base, "device blocks leaked: %ld", fakehip::live_blocks.load() - base);
    for (long k = 0; k <= total; ++k) {
        fakehip::malloc_calls = 0;
        fakehip::fail_after = k;
        const int rc = run_sequence(p);
        fakehip::fail_after = -1;
        CHECK(rc == 0, "device allocation %ld failing: unexpected status %d", k, rc);
        CHECK(fakehip::live_blocks.load() == base, "device allocation %ld failing: %ld blocks leaked", k,
              fakehip::live_blocks.load() - base);
    }
    std::printf("nomem: %ld device allocations, each made to fail in turn\n", total);
    // host allocations: operator new throws at the k-th call from now on
    for (long k = 0; k < 400; k += 3) {
        const int rc = run_sequence(p, k);
        CHECK(rc == 0, "host allocation %ld failing: unexpected status %d", k, rc);
    }
    std::printf("nomem: host allocations 0..399 (every third) made to fail\n");
}

static void scenario_threads()
{
    Problem p = make_problem(17);
    mesh_sdd_ctx *ctx = nullptr;
    CHECK(mesh_sdd_ctx_create(0, 0, nullptr, &ctx) == MESH_SDD_OK, "ctx_create");
    if (!ctx) return;
    std::atomic<bool> stop{false};
    std::atomic<int> done{0}, cancelled{0};
    std::thread watcher([&] {
        mesh_sdd_stats s;
        std::memset(&s, 0, sizeof s);
        s.struct_size = sizeof s;
        while (!stop) CHECK(mesh_sdd_ctx_stats(ctx, &s) == MESH_SDD_OK, "stats");
    });
    std::vector<std::thread> clients;
    for (int c = 0; c < 6; ++c)
        clients.emplace_back([&, c] {
            mesh_sdd *h = nullptr;
            mesh_sdd_desc d = make_desc(17, c % 2 ? 2 : 4, c == 5 ? MESH_SDD_FP64 : MESH_SDD_FP32, (uint32_t)c);
            if (mesh_sdd_create(ctx, &d, &h) != MESH_SDD_OK) {
                CHECK(false, "create in client %d", c);
                return;
            }
            CHECK(mesh_sdd_set_monitor(h, p.rho.data(), 0) == MESH_SDD_OK, "set_monitor");
            const int m = mesh_sdd_num_interface_nodes(h);
            for (int r = 0; r < 25; ++r) {
                mesh_sdd_step st = make_step(p, 64 + 64 * (r % 4), 0);
                Out o(m);
                mesh_sdd_ticket t = 0;
                if (mesh_sdd_submit(h, &st, &t) != MESH_SDD_OK) {
                    CHECK(false, "submit");
                    continue;
                }
                if (r % 5 == 1 && mesh_sdd_cancel(ctx, t) == MESH_SDD_OK) {
                    ++cancelled;
                    CHECK(mesh_sdd_poll(ctx, t, &o.r) == MESH_SDD_E_CANCELLED, "poll of a cancelled request");
                    continue;
                }
                int rc;
                if (r % 3 == 0) {
                    while ((rc = mesh_sdd_poll(ctx, t, &o.r)) == MESH_SDD_PENDING) std::this_thread::yield();
                } else {
                    rc = mesh_sdd_wait(ctx, t, &o.r, -1);
                }
                CHECK(rc == MESH_SDD_OK, "request %d of client %d: %d", r, c, rc);
                ++done;
            }
            while (mesh_sdd_destroy(h) == MESH_SDD_E_STATE) std::this_thread::yield();
        });
    for (auto &t : clients) t.join();
    stop = true;
    watcher.join();
    CHECK(mesh_sdd_ctx_destroy(ctx) == MESH_SDD_OK, "ctx_destroy");
    std::printf("threads: %d requests completed, %d cancelled\n", done.load(), cancelled.load());
    CHECK(done + cancelled == 150, "every request ended (%d)", done + cancelled);
}

// ---------------------------------------------------------------------------
static void scenario_split()
{
    mesh_sdd_ctx *ctx = nullptr;
    CHECK(mesh_sdd_ctx_create(0, 0, nullptr, &ctx) == MESH_SDD_OK, "ctx_create");
    if (!ctx) return;
    Problem p = make_problem(17);
    // 29 nodes x 40 chunks of 128 paths = 1160 items per request: two fit
    // under the limit of 3000, the third starts a second launch, the fourth
    // joins it; then a lone request of 29 x 104 = 3016 items is refused
    std::vector<mesh_sdd *> hs(4, nullptr);
    for (int q = 0; q < 4; ++q) {
        mesh_sdd_desc d = make_desc(17, 2, MESH_SDD_FP32, (uint32_t)q);
        CHECK(mesh_sdd_create(ctx, &d, &hs[q]) == MESH_SDD_OK, "create %d", q);
        if (hs[q]) CHECK(mesh_sdd_set_monitor(hs[q], p.rho.data(), 0) == MESH_SDD_OK, "set_monitor %d", q);
    }
    for (mesh_sdd *h : hs)
        if (!h) return;
    const int m = mesh_sdd_num_interface_nodes(hs[0]);
    std::vector<mesh_sdd_step> steps(4, make_step(p, 128 * 40, 0));
    std::vector<Out> outs;
    for (int q = 0; q < 4; ++q) outs.emplace_back(m);
    std::vector<mesh_sdd_result> res;
    for (auto &o : outs) res.push_back(o.r);
    int32_t status[4] = {9, 9, 9, 9};
    const int before = msdd::g_fp32_launches.load();
    CHECK(mesh_sdd_solve_batch(hs.data(), steps.data(), res.data(), 4, status) == MESH_SDD_OK, "split batch");
    for (int q = 0; q < 4; ++q) CHECK(status[q] == MESH_SDD_OK, "status %d = %d", q, status[q]);
    CHECK(msdd::g_fp32_launches.load() - before == 2, "launches %d, want 2", msdd::g_fp32_launches.load() - before);
    mesh_sdd_step big = make_step(p, 128 * 104, 0);
    Out ob(m);
    CHECK(mesh_sdd_solve_interfaces(hs[0], &big, &ob.r) == MESH_SDD_E_INVAL, "a request above the launch limit");
    for (mesh_sdd *h : hs) mesh_sdd_destroy(h);
    mesh_sdd_ctx_destroy(ctx);
}

int main(int argc, char **argv)
{
    const std::string what = argc > 1 ? argv[1] : "abi";
    const char *tmp = argc > 2 ? argv[2] : "/tmp";
    if (what == "abi")
        scenario_abi(tmp);
    else if (what == "nomem")
        scenario_nomem();
    else if (what == "threads")
        scenario_threads();
    else if (what == "split")
        scenario_split();
    else {
        std::fprintf(stderr, "unknown scenario %s\n", what.c_str());
        return 2;
    }
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("%s: all checks passed\n", what.c_str());
    return 0;
}
