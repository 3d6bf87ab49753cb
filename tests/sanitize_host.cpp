// Host-side checks of the library under AddressSanitizer + UndefinedBehavior-
// Sanitizer or ThreadSanitizer (built by tests/test_sanitizers.py; no GPU is
// used): layouts of every kind, the threaded BVH builder on awkward scenes,
// argument validation, and the serving dispatcher thread in its simulated
// mode with requests submitted from two threads at once.  Exits non-zero on
// a failed check; the sanitizers abort on the first report.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "vafr.h"

static int g_fail = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                   \
        }                                                               \
    } while (0)

static uint32_t lcg(uint32_t& s) { return s = s * 1664525u + 1013904223u; }
static float unit(uint32_t& s) { return (float)(lcg(s) >> 8) * (1.0f / 16777216.0f); }

static void layouts() {
    const vafr_display d{1920, 1080, 100.0, 100.0};
    vafr_layout L = nullptr;
    CHECK(vafr_lp_layout(&d, nullptr, &L) == VAFR_OK);
    vafr_dims dims;
    CHECK(vafr_layout_dims(L, &dims) == VAFR_OK);
    CHECK(dims.n_cols == 901 && dims.n_texels == 1063314);
    const int32_t* nr;
    const int64_t* off;
    const float* dxy;
    CHECK(vafr_layout_tables(L, &nr, &off, &dxy) == VAFR_OK);
    int64_t sum = 0;
    for (int i = 0; i < dims.n_cols; ++i) sum += nr[i];
    CHECK(sum == dims.n_texels && off[dims.n_cols] == dims.n_texels);
    double r2 = 0;
    for (int64_t k = 0; k < 2 * dims.n_texels; ++k) r2 += (double)dxy[k] * dxy[k];
    CHECK(std::isfinite(r2));
    int64_t ws = 0;
    CHECK(vafr_rep_workspace_bytes(L, &ws) == VAFR_OK && ws > 0);
    vafr_layout_destroy(L);
    // device-adapted and anisotropic curves
    double e[32], c[32];
    int32_t n = 0;
    for (double cap : {9.0, 18.0, 40.0, 0.5}) {
        CHECK(vafr_acuity_capped(nullptr, cap, e, c, 32, &n) == VAFR_OK);
        const double ae[2] = {0.0, 30.0}, ad[2] = {1.0, 0.5};
        vafr_acuity a{n, e, c, 60.0, 2, ae, ad};
        CHECK(vafr_lp_layout(&d, &a, &L) == VAFR_OK);
        vafr_layout_destroy(L);
    }
    CHECK(vafr_acuity_capped(nullptr, 9.0, e, c, 2, &n) == VAFR_E_ARG);
    // invalid curves and displays
    const double be[3] = {0.0, 20.0, 10.0}, bc[3] = {40.0, 10.0, 6.0};
    vafr_acuity bad{3, be, bc, 60.0, 0, nullptr, nullptr};
    CHECK(vafr_lp_layout(&d, &bad, &L) == VAFR_E_ARG);
    const vafr_display bd{0, 1080, 100.0, 100.0};
    CHECK(vafr_lp_layout(&bd, nullptr, &L) == VAFR_E_ARG);
    CHECK(vafr_lp_layout(nullptr, nullptr, &L) == VAFR_E_ARG);
    // dense comparison layouts, tiny and large displays
    for (const vafr_display& dd : {vafr_display{7, 5, 100.0, 100.0}, vafr_display{7680, 4320, 100.0, 100.0},
                                   vafr_display{11520, 6480, 100.0, 100.0}}) {
        CHECK(lmfr_lp_layout(&dd, 1.8, 4.0, &L) == VAFR_OK);
        CHECK(vafr_layout_tables(L, &nr, &off, &dxy) == VAFR_OK && dxy == nullptr);
        vafr_layout_destroy(L);
        CHECK(lafr_lp_layout(&dd, 2.2, 0.25, 0.78, 0.9, &L) == VAFR_OK);
        vafr_layout_destroy(L);
    }
    CHECK(lmfr_lp_layout(&d, 0.5, 4.0, &L) == VAFR_E_ARG);
    CHECK(lafr_lp_layout(&d, 1.8, 1.5, 0.85, 0.7, &L) == VAFR_E_ARG);
}

static vafr_scene make_scene(const std::vector<float>& v, const std::vector<int32_t>& t, int expect = VAFR_OK) {
    vafr_scene s = nullptr;
    const int rc = vafr_scene_create(v.data(), (int64_t)v.size() / 3, t.data(), (int64_t)t.size() / 3, &s);
    CHECK(rc == expect);
    if (rc == VAFR_OK) {
        vafr_scene_info info;
        CHECK(vafr_scene_get_info(s, &info) == VAFR_OK);
        CHECK(info.n_tris == (int64_t)t.size() / 3);
        std::vector<float> nodes(16 * (size_t)std::max<int64_t>(info.n_nodes, 1));
        std::vector<int32_t> order(std::max<size_t>(t.size() / 3, 1));
        CHECK(vafr_scene_export(s, nodes.data(), order.data()) == VAFR_OK);
        std::vector<char> seen(t.size() / 3, 0);
        for (size_t k = 0; k < t.size() / 3; ++k) {
            CHECK(order[k] >= 0 && (size_t)order[k] < seen.size() && !seen[order[k]]);
            if (order[k] >= 0 && (size_t)order[k] < seen.size()) seen[order[k]] = 1;
        }
    }
    return s;
}

static void scenes() {
    uint32_t seed = 7;
    // random soup
    std::vector<float> v;
    std::vector<int32_t> t;
    for (int k = 0; k < 3 * 20000; ++k) {
        for (int c = 0; c < 3; ++c) v.push_back(2.0f * unit(seed) - 1.0f);
        t.push_back(k);
    }
    vafr_scene_destroy(make_scene(v, t));
    // heightfield grid with shared vertices
    const int nx = 256, nz = 128;
    v.clear();
    t.clear();
    for (int z = 0; z <= nz; ++z)
        for (int x = 0; x <= nx; ++x) {
            v.push_back(-2.0f + 4.0f * x / nx);
            v.push_back(-0.6f + 0.05f * std::sin(0.3f * x) * std::cos(0.2f * z));
            v.push_back(-1.0f + 2.0f * z / nz);
        }
    for (int z = 0; z < nz; ++z)
        for (int x = 0; x < nx; ++x) {
            const int a = z * (nx + 1) + x, b = a + 1, c = a + nx + 1, d = c + 1;
            t.insert(t.end(), {a, b, d, a, d, c});
        }
    vafr_scene_destroy(make_scene(v, t));
    // coincident, degenerate and tiny triangles (deep trees, zero extents)
    v.clear();
    t.clear();
    for (int k = 0; k < (1 << 14); ++k) {
        v.insert(v.end(), {-8.0f, -8.0f, 1.0f, 8.0f, -8.0f, 1.0f, 0.0f, 8.0f, 1.0f});
        t.insert(t.end(), {3 * k, 3 * k + 1, 3 * k + 2});
    }
    for (int k = 0; k < 1000; ++k) {
        const int b = (int)v.size() / 3;
        const float x = unit(seed);
        v.insert(v.end(), {x, x, x, x, x, x, x + 1e-7f, x, x});
        t.insert(t.end(), {b, b + 1, b + 2});
    }
    vafr_scene_destroy(make_scene(v, t));
    // empty scene, out-of-range index, non-finite vertex
    vafr_scene_destroy(make_scene({}, {}));
    make_scene({0, 0, 0, 1, 0, 0, 0, 1, 0}, {0, 1, 3}, VAFR_E_ARG);
    make_scene({0, 0, 0, NAN, 0, 0, 0, 1, 0}, {0, 1, 2}, VAFR_E_ARG);
    // several builds at once (the builder's own threads run inside each)
    std::vector<std::thread> th;
    for (int i = 0; i < 3; ++i)
        th.emplace_back([&v, &t] {
            vafr_scene s = nullptr;
            if (vafr_scene_create(v.data(), (int64_t)v.size() / 3, t.data(), (int64_t)t.size() / 3, &s) == VAFR_OK)
                vafr_scene_destroy(s);
        });
    for (auto& x : th) x.join();
}

static void serving() {
    vafr_server_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.max_views_per_launch = 16;
    cfg.max_inflight = 2;
    cfg.n_streams = 1;
    cfg.max_queue = 48;
    cfg.hbm_budget_bytes = (int64_t)1 << 30;
    cfg.batch = vafr_batch_config{128, 8, 1};
    cfg.simulate = 1;
    cfg.sim_ms_per_launch = 0.2;
    cfg.sim_ms_per_mray = 0.3;
    cfg.sim_ms_per_mpix = 0.01;
    cfg.frame_budget_ms = 6.0;
    cfg.latest_only = 1;
    vafr_server srv = nullptr;
    CHECK(vafr_server_create(&cfg, &srv) == VAFR_OK);
    const vafr_display d{1280, 720, 100.0, 100.0};
    vafr_layout L = nullptr;
    CHECK(vafr_lp_layout(&d, nullptr, &L) == VAFR_OK);
    vafr_headset hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.layout = L;
    for (int e = 0; e < 2; ++e) {
        hs.camera[e].right[0] = hs.camera[e].up[1] = hs.camera[e].forward[2] = 1.0f;
        hs.camera[e].eye[0] = e ? 0.032f : -0.032f;
    }
    hs.shading.light_dir[1] = 1.0f;
    for (int h = 0; h < 4; ++h) {
        int32_t id = -1;
        CHECK(vafr_server_add_headset(srv, &hs, &id) == VAFR_OK && id == h);
    }
    std::atomic<int> done{0};
    std::atomic<int64_t> finished{0};
    auto submitter = [&](int base) {
        for (int f = 0; f < 400; ++f) {
            vafr_request r;
            std::memset(&r, 0, sizeof(r));
            r.headset = base + (f & 1);
            r.frame = (uint32_t)f;
            r.gaze = vafr_gaze{640.0 + f % 7, 360.0 - f % 5};
            r.user_tag = (uint64_t)(base * 1000 + f);
            (void)vafr_server_submit(srv, &r);
            if (f % 16 == 0) std::this_thread::sleep_for(std::chrono::microseconds(300));
        }
        ++done;
    };
    std::thread a(submitter, 0), b(submitter, 2);
    std::vector<vafr_result> res(64);
    for (;;) {
        int32_t n = 0;
        CHECK(vafr_server_poll(srv, res.data(), (int32_t)res.size(), &n) == VAFR_OK);
        for (int i = 0; i < n; ++i) {
            if (res[i].status == VAFR_OK) CHECK(vafr_server_release(srv, res[i].slot) == VAFR_OK);
            ++finished;
        }
        vafr_server_stats st;
        CHECK(vafr_server_get_stats(srv, &st) == VAFR_OK);
        if (done.load() == 2 && st.waiting == 0 && st.inflight == 0 && finished.load() + st.refused >= st.submitted)
            break;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    a.join();
    b.join();
    vafr_server_stats st;
    CHECK(vafr_server_get_stats(srv, &st) == VAFR_OK);
    CHECK(st.submitted == 800 && st.completed > 0);
    CHECK(st.completed + st.dropped == st.submitted - st.refused);
    CHECK(vafr_server_wait_idle(srv, 5000) == VAFR_OK);
    vafr_server_destroy(srv);
    vafr_layout_destroy(L);
    std::printf("serving: %lld submitted, %lld completed, %lld late, %lld superseded, %lld refused, %lld launches\n",
                (long long)st.submitted, (long long)st.completed, (long long)st.late, (long long)st.superseded,
                (long long)st.refused, (long long)st.launches);
}

// A simulated device that stops making progress: the watchdog gives up the
// launched work while a second thread keeps submitting.
static void stall() {
    vafr_server_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.max_views_per_launch = 4;
    cfg.max_inflight = 2;
    cfg.n_streams = 1;
    cfg.max_queue = 16;
    cfg.hbm_budget_bytes = (int64_t)1 << 30;
    cfg.batch = vafr_batch_config{128, 8, 1};
    cfg.simulate = 1;
    cfg.sim_ms_per_launch = 60000.0;
    cfg.watchdog_ms = 30.0;
    vafr_server srv = nullptr;
    CHECK(vafr_server_create(&cfg, &srv) == VAFR_OK);
    const vafr_display d{640, 360, 100.0, 100.0};
    vafr_layout L = nullptr;
    CHECK(vafr_lp_layout(&d, nullptr, &L) == VAFR_OK);
    vafr_headset hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.layout = L;
    for (int e = 0; e < 2; ++e) hs.camera[e].right[0] = hs.camera[e].up[1] = hs.camera[e].forward[2] = 1.0f;
    hs.shading.light_dir[1] = 1.0f;
    int32_t id = -1;
    CHECK(vafr_server_add_headset(srv, &hs, &id) == VAFR_OK);
    std::atomic<int64_t> accepted{0};
    std::thread sub([&] {
        for (int f = 0; f < 200; ++f) {
            vafr_request r;
            std::memset(&r, 0, sizeof(r));
            r.frame = (uint32_t)f;
            r.gaze = vafr_gaze{320.0, 180.0};
            if (vafr_server_submit(srv, &r) == VAFR_OK) ++accepted;
            std::this_thread::sleep_for(std::chrono::microseconds(500));
        }
    });
    sub.join();
    CHECK(vafr_server_wait_idle(srv, 5000) == VAFR_OK);   // the watchdog empties the queues
    int64_t timed_out = 0;
    std::vector<vafr_result> res(64);
    for (int i = 0; i < 400; ++i) {
        int32_t n = 0;
        const int rc = vafr_server_poll(srv, res.data(), (int32_t)res.size(), &n);
        for (int k = 0; k < n; ++k) {
            CHECK(res[k].status == VAFR_E_TIMEOUT && res[k].slot == 0);
            ++timed_out;
        }
        if (n == 0) {
            CHECK(rc == VAFR_E_TIMEOUT);
            break;
        }
    }
    vafr_server_stats st;
    CHECK(vafr_server_get_stats(srv, &st) == VAFR_OK);
    CHECK(st.stalled > 0 && st.stalled == timed_out && st.completed == 0 && st.inflight == 0);
    CHECK(st.dropped == accepted.load());
    vafr_server_destroy(srv);
    vafr_layout_destroy(L);
    std::printf("stall: %lld accepted, %lld timed out\n", (long long)accepted.load(), (long long)timed_out);
}

int main(int argc, char** argv) {
    const char* what = argc > 1 ? argv[1] : "all";
    if (!std::strcmp(what, "all") || !std::strcmp(what, "layouts")) layouts();
    if (!std::strcmp(what, "all") || !std::strcmp(what, "scenes")) scenes();
    if (!std::strcmp(what, "all") || !std::strcmp(what, "serving")) serving();
    if (!std::strcmp(what, "all") || !std::strcmp(what, "stall")) stall();
    std::printf("%s: %d failed checks\n", what, g_fail);
    return g_fail ? 1 : 0;
}
