// CPU test of the library's host logic on a fake device (fake_device.cpp), built with
// -fsanitize=address,undefined by tests/test_host_logic.py:
//   the serving arena's first-fit allocator against a granule-by-granule model;
//   the tile planners: every plan covers its level exactly once, within the kernel's capacity;
//   the batched stage choice fits every level of the stage;
//   whole solves on the toy device: a pair solved alone, in a batch (table and work-queue orders,
//   several K) and served in randomised submit / step / poll orders gives bitwise the same flow
//   and energy, while the server keeps its memory budget, its slot limit and its ticket contract.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "../../include/flow.h"
#include "multi.hpp"
#include "runtime.hpp"

long fake_device_launches();
size_t fake_device_live_allocations();

using namespace flowmi;

static int g_fail = 0;
#define CHECK(cond, ...)                                                  \
    do {                                                                  \
        if (!(cond)) {                                                    \
            std::fprintf(stderr, "CHECK failed %s:%d: %s -- ", __FILE__, __LINE__, #cond); \
            std::fprintf(stderr, __VA_ARGS__);                            \
            std::fprintf(stderr, "\n");                                   \
            if (++g_fail > 20) std::exit(1);                              \
        }                                                                 \
    } while (0)
#define OK(expr)                                                          \
    do {                                                                  \
        flow_status _s = (expr);                                          \
        if (_s != FLOW_OK) {                                              \
            std::fprintf(stderr, "%s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #expr, (int)_s, flow_last_error()); \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

// ------------------------------------------------------------------ first-fit allocator
static void test_range_alloc(std::mt19937& rng) {
    for (int round = 0; round < 40; ++round) {
        const size_t gran = 256, cap = gran * (64 + rng() % 512);
        RangeAlloc ra;
        ra.reset(cap);
        std::vector<int> owner(cap / gran, -1);      // model: which allocation holds each granule
        std::map<int, std::pair<size_t, size_t>> live;
        int next = 0;
        for (int op = 0; op < 600; ++op) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t n = gran * (1 + rng() % 40);
                size_t off = 0;
                const bool got = ra.alloc(n, off);
                // first fit: the lowest offset whose free run holds n (the model's answer)
                size_t want = SIZE_MAX;
                for (size_t g = 0, run = 0; g < owner.size(); ++g) {
                    run = owner[g] < 0 ? run + 1 : 0;
                    if (run * gran >= n) { want = (g + 1) * gran - run * gran; break; }
                }
                CHECK(got == (want != SIZE_MAX), "alloc of %zu: got %d, model %d", n, (int)got, (int)(want != SIZE_MAX));
                if (got) {
                    CHECK(off == want, "first fit at %zu, model %zu", off, want);
                    CHECK(off % gran == 0 && off + n <= cap, "range [%zu, %zu) of %zu", off, off + n, cap);
                    for (size_t g = off / gran; g < (off + n) / gran; ++g) {
                        CHECK(owner[g] < 0, "granule %zu handed out twice", g);
                        owner[g] = next;
                    }
                    live[next++] = {off, n};
                }
            } else {
                auto it = live.begin();
                std::advance(it, rng() % live.size());
                ra.release(it->second.first, it->second.second);
                for (size_t g = it->second.first / gran; g < (it->second.first + it->second.second) / gran; ++g) owner[g] = -1;
                live.erase(it);
            }
            // free list: sorted, disjoint, merged, and exactly the model's free granules
            size_t prev_end = 0, free_bytes = 0;
            bool first = true;
            for (auto& kv : ra.free_) {
                CHECK(kv.second > 0 && kv.first + kv.second <= cap, "free range [%zu, +%zu)", kv.first, kv.second);
                CHECK(first || kv.first > prev_end, "free ranges touch or overlap at %zu", kv.first);
                for (size_t g = kv.first / gran; g < (kv.first + kv.second) / gran; ++g)
                    CHECK(owner[g] < 0, "granule %zu both free and held", g);
                prev_end = kv.first + kv.second;
                free_bytes += kv.second;
                first = false;
            }
            size_t model_free = 0;
            for (int o : owner) model_free += o < 0 ? gran : 0;
            CHECK(free_bytes == model_free, "free bytes %zu, model %zu", free_bytes, model_free);
        }
    }
}

// ------------------------------------------------------------------ tile planners
static void check_cover(const std::vector<TbTile>& tiles, int H, int W, const char* what) {
    std::vector<int> hit((size_t)H * W, 0);
    for (const TbTile& t : tiles) {
        CHECK(t.y0 >= 0 && t.x0 >= 0 && t.th > 0 && t.tw > 0 && t.y0 + t.th <= H && t.x0 + t.tw <= W,
              "%s: tile (%d, %d, %d, %d) outside %dx%d", what, t.y0, t.x0, t.th, t.tw, H, W);
        for (int i = t.y0; i < std::min(H, t.y0 + t.th); ++i)
            for (int j = t.x0; j < std::min(W, t.x0 + t.tw); ++j) hit[(size_t)i * W + j]++;
    }
    for (size_t k = 0; k < hit.size(); ++k)
        if (hit[k] != 1) {
            CHECK(false, "%s: pixel %zu of %dx%d covered %d times", what, k, H, W, hit[k]);
            return;
        }
}

static void test_planners(std::mt19937& rng) {
    const int nts[] = {256, 1024, 1025, 513, 257, 1026, 514, 2049, 3073, 4097};
    for (int c = 0; c < 1500; ++c) {
        const int H = 2 + rng() % (rng() % 8 ? 300 : 2500), W = 2 + rng() % (rng() % 8 ? 300 : 2500);
        const bool hw = rng() % 2;
        const int nt = nts[rng() % 10], K = 1 + rng() % 16;
        const int ew = rng() % 3 ? 0 : 16 + rng() % 300;
        const LevelTbPlan P = plan_tiles(H, W, hw, nt, K, ew);
        if (!P.tb) continue;
        std::vector<TbTile> tiles;
        append_tiles(P, 7, H, W, tiles);
        CHECK(!tiles.empty() && tiles[0].level == 7, "tiles name their level");
        check_cover(tiles, H, W, "plan_tiles");
        CHECK(P.K >= 1 && P.K <= K, "K %d of %d", P.K, K);
        for (const TbTile& t : tiles) {
            const int ey0 = std::max(t.y0 - tb_halo_lo(P.K), 0), ex0 = std::max(t.x0 - tb_halo_lo(P.K), 0);
            const int ey1 = std::min(t.y0 + t.th + tb_halo_hi(P.K), H), ex1 = std::min(t.x0 + t.tw + tb_halo_hi(P.K), W);
            CHECK(tb_fits(hw, nt, ey1 - ey0, ex1 - ex0), "extended tile %dx%d beyond the shape of code %d (H %d W %d K %d)",
                  ey1 - ey0, ex1 - ex0, nt, H, W, P.K);
        }
        // the full plan of a mode (with the balancing of tile heights) covers the level as well
        const int modes[] = {2, 3, 4, 6, 7, 8, 9, 12, 13, 14};
        const LevelTbPlan Q = plan_level(H, W, hw, 50, modes[rng() % 10], K, ew);
        if (Q.tb) {
            std::vector<TbTile> tq;
            append_tiles(Q, 0, H, W, tq);
            check_cover(tq, H, W, "plan_level");
        }
        // pDR / ALG1 tiles
        const int halo = 3 * (1 + rng() % 4);
        const int pnt[] = {512, 1024, 2048, 513, 4098, 6145, 3074, 2050};
        const PdrTbPlan R = plan_pd_tiles(H, W, hw, halo, 1 + rng() % 4, rng() % 2 ? 0 : 32 + rng() % 64,
                                          pnt[rng() % 8]);
        if (R.tb && !R.resident) {
            CHECK(R.th >= 2 && (R.tw >= 8 || R.tw == W), "pDR tile %dx%d of a level %d wide", R.th, R.tw, W);
            const int ext_w = std::min(W, R.tw + halo), ext_h = std::min(H, R.th + halo);
            CHECK(pd_fits(hw, R.nt, ext_h, ext_w), "pDR extended tile %dx%d (code %d)", ext_h, ext_w, R.nt);
        }
    }
    // batched stages: the choice fits every level, and each level's tiles cover it
    for (int c = 0; c < 200; ++c) {
        Shapes s;
        const int n = 1 + rng() % 6;
        for (int k = 0; k < n; ++k) s.emplace_back(2 + rng() % 800, 2 + rng() % 1400);
        const bool hw = rng() % 2;
        StageChoice ch;
        ch.K = 1 + rng() % 20;
        ch.ew = rng() % 2 ? 64 : 16 + rng() % 200;
        ch.order = rng() % 2;
        const StageChoice f = fit_stage_choice(ch, s, hw);
        CHECK(f.K >= 1 && f.K <= ch.K, "fitted K %d of %d", f.K, ch.K);
        CHECK(shapes_fit(s, hw, f.K, f.ew) || f.K == 1, "fitted choice K %d ew %d does not fit", f.K, f.ew);
        const StageChoice d = default_stage_choice(s, hw, 50);
        CHECK(d.K >= 1, "built-in K %d", d.K);
        for (auto& x : s) {
            const LevelTbPlan T = plan_tiles(x.first, x.second, hw, kBatchNt, std::min(f.K, 64), f.ew);
            CHECK(T.tb && T.th > 0 && T.tw > 0, "stage level %dx%d has no tiles for K %d ew %d (from K %d ew %d)",
                  x.first, x.second, f.K, f.ew, ch.K, ch.ew);
            if (!T.tb) continue;
            std::vector<TbTile> t;
            level_tiles(x.first, x.second, hw, f, 3, t);
            check_cover(t, x.first, x.second, "level_tiles");
        }
    }
}

// ------------------------------------------------------------------ whole solves on the toy device
struct Frame {
    int H, W, levels;
    float *I0, *I1;        // device (fake), pitch W
};
struct Out {
    std::vector<float> u, v;
    double energy = 0, gap = 0;
    bool operator==(const Out& o) const {
        return u == o.u && v == o.v && std::memcmp(&energy, &o.energy, sizeof(double)) == 0 &&
               std::memcmp(&gap, &o.gap, sizeof(double)) == 0;
    }
};

static Frame make_frame(std::mt19937& rng, int H, int W, int levels) {
    Frame f{H, W, levels, nullptr, nullptr};
    hipMalloc(&f.I0, sizeof(float) * H * W);
    hipMalloc(&f.I1, sizeof(float) * H * W);
    for (int k = 0; k < H * W; ++k) {
        f.I0[k] = (float)(rng() % 256);
        f.I1[k] = (float)(rng() % 256);
    }
    return f;
}

static flow_params params(int levels) {
    flow_params p;
    flow_params_default(&p);
    p.levels = levels;
    p.warps = 3;
    p.iters = 12;
    return p;
}

static Out read_out(const Frame& f, float* u, float* v, const flow_result& r) {
    Out o;
    o.u.assign(u, u + f.H * f.W);
    o.v.assign(v, v + f.H * f.W);
    o.energy = r.energy;
    o.gap = r.gap;
    for (float x : o.u) CHECK(std::isfinite(x), "non-finite flow");
    CHECK(std::isfinite(r.energy), "non-finite energy");
    return o;
}

static Out solve_alone(flow_ctx* ctx, const Frame& f, int use_graph) {
    float *u, *v;
    hipMalloc(&u, sizeof(float) * f.H * f.W);
    hipMalloc(&v, sizeof(float) * f.H * f.W);
    flow_params p = params(f.levels);
    p.use_graph = use_graph;
    flow_result r{};
    OK(flow_solve(ctx, f.I0, f.I1, f.H, f.W, f.W, &p, u, v, f.W, &r, nullptr));
    Out o = read_out(f, u, v, r);
    hipFree(u);
    hipFree(v);
    return o;
}

static std::vector<Out> solve_batch(flow_ctx* ctx, const std::vector<Frame>& fs, int use_graph) {
    std::vector<flow_pair> ps(fs.size());
    std::vector<flow_result> rs(fs.size());
    std::vector<float*> bufs;
    for (size_t k = 0; k < fs.size(); ++k) {
        float *u, *v;
        hipMalloc(&u, sizeof(float) * fs[k].H * fs[k].W);
        hipMalloc(&v, sizeof(float) * fs[k].H * fs[k].W);
        bufs.push_back(u);
        bufs.push_back(v);
        ps[k] = flow_pair{fs[k].I0, fs[k].I1, fs[k].H, fs[k].W, fs[k].W, u, v, fs[k].W, &rs[k], fs[k].levels};
    }
    flow_params p = params(5);
    p.use_graph = use_graph;
    OK(flow_solve_batched(ctx, (int)fs.size(), ps.data(), &p, nullptr));
    std::vector<Out> out;
    for (size_t k = 0; k < fs.size(); ++k) out.push_back(read_out(fs[k], ps[k].u, ps[k].v, rs[k]));
    for (float* b : bufs) hipFree(b);
    return out;
}

static void test_solves(std::mt19937& rng) {
    flow_ctx* ctx = nullptr;
    OK(flow_create(&ctx, 0, 0));
    std::vector<Frame> fs;
    for (int k = 0; k < 9; ++k) {
        const int H = 12 + rng() % 90, W = 12 + rng() % 130;
        int lv = 1;
        while (lv < 4 && std::min(H, W) >> lv >= 4) ++lv;
        fs.push_back(make_frame(rng, H, W, lv));
    }
    fs.push_back(make_frame(rng, 150, 10, 2));      // levels narrower than 8 pixels (75 x 5, 5 x 100)
    fs.push_back(make_frame(rng, 9, 200, 2));
    // reference: each pair alone with small 1024-thread tiles at every level (the batched kernel)
    OK(flow_tune_set("tb_mode", 4));
    std::vector<Out> ref;
    for (auto& f : fs) ref.push_back(solve_alone(ctx, f, 0));
    CHECK(solve_alone(ctx, fs[0], 1) == ref[0], "graph replay differs from direct launches");
    OK(flow_tune_set("tb_mode", 1));                 // one-pass kernel: one launch per iteration
    CHECK(solve_alone(ctx, fs[1], 0) == ref[1], "one-pass plan differs from tiles");
    OK(flow_tune_set("tb_mode", 0));
    CHECK(solve_alone(ctx, fs[2], 1) == ref[2], "built-in plan differs from tiles");

    // batches: random subsets, both orders, several K, direct and replayed
    for (int round = 0; round < 8; ++round) {
        std::vector<Frame> sub;
        std::vector<int> idx;
        for (size_t k = 0; k < fs.size(); ++k)
            if (rng() % 2) { sub.push_back(fs[k]); idx.push_back((int)k); }
        if (sub.empty()) continue;
        const int bnt[] = {0, 1025, 2049, 3073, 4097};
        OK(flow_tune_set("batch_order", (int)(rng() % 2)));
        OK(flow_tune_set("batch_k", (int)(rng() % 4 == 0 ? 0 : 1 + rng() % 13)));
        OK(flow_tune_set("batch_nt", bnt[rng() % 5]));
        const std::vector<Out> got = solve_batch(ctx, sub, (int)(rng() % 2));
        for (size_t i = 0; i < sub.size(); ++i)
            CHECK(got[i] == ref[idx[i]], "batched pair %d (round %d) differs from alone", idx[i], round);
    }
    OK(flow_tune_set("batch_order", -1));
    OK(flow_tune_set("batch_k", 0));
    OK(flow_tune_set("batch_nt", 0));

    // serving: randomised submit / step / poll orders under a budget that holds two or three pairs
    for (int round = 0; round < 10; ++round) {
        OK(flow_tune_set("serve_graph", (int)(rng() % 2)));
        OK(flow_tune_set("batch_nt", rng() % 2 ? 0 : 3073));
        uint64_t big = 0;
        for (auto& f : fs) {
            uint64_t b = 0;
            flow_params p = params(f.levels);
            OK(flow_working_set_bytes(f.H, f.W, &p, f.levels, &b));
            big = std::max(big, b);
        }
        const size_t budget = (size_t)big * (2 + rng() % 2);
        const int max_active = 1 + (int)(rng() % 4);
        flow_params p = params(4);
        flow_server* srv = nullptr;
        OK(flow_server_create(ctx, &p, budget, max_active, nullptr, &srv));
        struct Sub { uint64_t t; int k; float *u, *v; flow_result r; bool collected = false; };
        std::vector<Sub*> subs;
        int n_sub = 0;
        for (int op = 0; op < 120; ++op) {
            const int what = (int)(rng() % 4);
            if (what == 0 && n_sub < 30) {
                Sub* s = new Sub();
                s->k = (int)(rng() % fs.size());
                const Frame& f = fs[s->k];
                hipMalloc(&s->u, sizeof(float) * f.H * f.W);
                hipMalloc(&s->v, sizeof(float) * f.H * f.W);
                flow_pair q{f.I0, f.I1, f.H, f.W, f.W, s->u, s->v, f.W, &s->r, f.levels};
                OK(flow_server_submit(srv, &q, &s->t));
                subs.push_back(s);
                ++n_sub;
            } else if (what == 1 || what == 2) {
                int32_t a = 0, qd = 0;
                OK(flow_server_step(srv, &a, &qd));
            } else if (!subs.empty()) {
                Sub* s = subs[rng() % subs.size()];
                int32_t done = 0;
                const flow_status st = flow_server_poll(srv, s->t, &done);
                if (s->collected) {
                    CHECK(st == FLOW_E_NOTFOUND, "a collected ticket polled again gives %d", (int)st);
                } else {
                    CHECK(st == FLOW_OK, "poll -> %d", (int)st);
                    if (done) {
                        s->collected = true;
                        CHECK(read_out(fs[s->k], s->u, s->v, s->r) == ref[s->k], "served pair %d differs from alone", s->k);
                    }
                }
            }
            flow_server_stats st{};
            OK(flow_server_get_stats(srv, &st));
            CHECK(st.bytes_in_use <= st.arena_bytes && st.peak_bytes_in_use <= st.arena_bytes,
                  "budget: %llu in use of %llu", (unsigned long long)st.bytes_in_use, (unsigned long long)st.arena_bytes);
            CHECK(st.active <= max_active && st.peak_active <= max_active, "slots: %d active of %d", st.active, max_active);
            CHECK(st.completed <= st.admitted && st.admitted <= st.submitted, "counters");
        }
        OK(flow_server_drain(srv));
        for (Sub* s : subs) {
            if (!s->collected) {
                int32_t done = 0;
                OK(flow_server_poll(srv, s->t, &done));
                CHECK(done == 1, "ticket not done after drain");
                CHECK(read_out(fs[s->k], s->u, s->v, s->r) == ref[s->k], "served pair %d differs from alone (drained)", s->k);
            }
            hipFree(s->u);
            hipFree(s->v);
            delete s;
        }
        flow_server_stats st{};
        OK(flow_server_get_stats(srv, &st));
        CHECK(st.completed == n_sub && st.active == 0 && st.queued == 0 && st.bytes_in_use == 0, "drained server");
        OK(flow_server_destroy(srv));
    }
    OK(flow_tune_set("serve_graph", 1));
    OK(flow_tune_set("batch_nt", 0));

    // a pair that can never fit the budget is refused at submit
    {
        flow_params p = params(2);
        flow_server* srv = nullptr;
        OK(flow_server_create(ctx, &p, 1 << 16, 2, nullptr, &srv));
        flow_pair q{fs[0].I0, fs[0].I1, fs[0].H, fs[0].W, fs[0].W, fs[0].I0, fs[0].I1, fs[0].W, nullptr, 2};
        uint64_t t = 0;
        CHECK(flow_server_submit(srv, &q, &t) == FLOW_E_NOMEM, "oversized pair admitted");
        OK(flow_server_destroy(srv));
    }
    for (auto& f : fs) {
        hipFree(f.I0);
        hipFree(f.I1);
    }
    OK(flow_destroy(ctx));
    CHECK(fake_device_live_allocations() == 0, "%zu device allocations leaked", fake_device_live_allocations());
}

// pDR and ALG1 solves under every kernel choice and K: each tile launch is checked by the fake
// device against its kernel's capacity (the large pDR tiles only without the w block)
static void test_pd_solves(std::mt19937& rng) {
    flow_ctx* ctx = nullptr;
    OK(flow_create(&ctx, 0, 0));
    for (int k = 0; k < 3; ++k) {
        const int H = 12 + rng() % 140, W = 12 + rng() % 160;
        int lv = 1;
        while (lv < 4 && std::min(H, W) >> lv >= 4) ++lv;
        Frame f = make_frame(rng, H, W, lv);
        float *u, *v;
        hipMalloc(&u, sizeof(float) * H * W);
        hipMalloc(&v, sizeof(float) * H * W);
        for (int mode : {0, 1, 5, 6, 10, 11, 12, 13, 14, 15})
            for (int K : {0, 1, 3}) {
                OK(flow_tune_set("pdr_mode", mode));
                OK(flow_tune_set("pdr_k", K));
                for (int scheme : {FLOW_PDR, FLOW_ALG1})
                    for (double beta : {0.0, 0.05}) {
                        flow_params p = params(lv);
                        p.scheme = scheme;
                        p.beta = beta;
                        p.use_graph = (int)(rng() % 2);
                        flow_result r{};
                        OK(flow_solve(ctx, f.I0, f.I1, H, W, W, &p, u, v, W, &r, nullptr));
                        read_out(f, u, v, r);
                    }
            }
        // ALG1 takes its kernel from per-level choices: every tile shape (wave-row 64 x 48 without w)
        for (int mode : {5, 6, 14, 15})
            for (int K : {0, 2, 5})
                for (double beta : {0.0, 0.05}) {
                    if (mode == 14 && beta > 0) continue;
                    flow_params p = params(lv);
                    p.scheme = FLOW_ALG1;
                    p.beta = beta;
                    int h = H, w = W;
                    for (int l = 0; l < lv; ++l, h = (h + 1) / 2, w = (w + 1) / 2)
                        OK(flow_tune_choice(ctx, h, w, beta > 0, p.iters, -1, mode, K, 0));
                    flow_result r{};
                    OK(flow_solve(ctx, f.I0, f.I1, H, W, W, &p, u, v, W, &r, nullptr));
                    read_out(f, u, v, r);
                }
        hipFree(u);
        hipFree(v);
        hipFree(f.I0);
        hipFree(f.I1);
    }
    OK(flow_tune_set("pdr_mode", 0));
    OK(flow_tune_set("pdr_k", 0));
    flow_destroy(ctx);
}

// Batched and served pDR and ALG1: every pair of random subsets, and every served pair, equals its
// plain tile solve, bit for bit
static void test_pd_batches(std::mt19937& rng) {
    flow_ctx* ctx = nullptr;
    OK(flow_create(&ctx, 0, 0));
    std::vector<Frame> fs;
    for (int k = 0; k < 5; ++k) {
        const int H = 12 + rng() % 140, W = 12 + rng() % 170;
        int lv = 1;
        while (lv < 4 && std::min(H, W) >> lv >= 4) ++lv;
        fs.push_back(make_frame(rng, H, W, lv));
    }
    fs.push_back(make_frame(rng, 150, 10, 2));
    for (int scheme : {FLOW_PDR, FLOW_ALG1})
        for (double beta : {0.0, 0.05}) {
            flow_params p = params(4);
            p.scheme = scheme;
            p.beta = beta;
            std::vector<Out> ref;
            for (auto& f : fs) {
                float *u, *v;
                hipMalloc(&u, sizeof(float) * f.H * f.W);
                hipMalloc(&v, sizeof(float) * f.H * f.W);
                flow_params q = p;
                q.levels = f.levels;
                flow_result r{};
                OK(flow_solve(ctx, f.I0, f.I1, f.H, f.W, f.W, &q, u, v, f.W, &r, nullptr));
                ref.push_back(read_out(f, u, v, r));
                hipFree(u);
                hipFree(v);
            }
            for (int round = 0; round < 3; ++round) {
                std::vector<flow_pair> ps;
                std::vector<flow_result> rs(fs.size());
                std::vector<int> idx;
                std::vector<float*> bufs;
                for (size_t k = 0; k < fs.size(); ++k) {
                    if (rng() % 3 == 0) continue;
                    float *u, *v;
                    hipMalloc(&u, sizeof(float) * fs[k].H * fs[k].W);
                    hipMalloc(&v, sizeof(float) * fs[k].H * fs[k].W);
                    bufs.push_back(u);
                    bufs.push_back(v);
                    idx.push_back((int)k);
                    ps.push_back(flow_pair{fs[k].I0, fs[k].I1, fs[k].H, fs[k].W, fs[k].W, u, v, fs[k].W, &rs[k],
                                           fs[k].levels});
                }
                if (ps.empty()) continue;
                flow_params q = p;
                q.use_graph = (int)(rng() % 2);
                // the last rounds take stage choices measured by the batched autotuner (any choice
                // changes speed only)
                if (round == 2) OK(flow_autotune_batched(ctx, (int)ps.size(), ps.data(), &q, nullptr));
                OK(flow_solve_batched(ctx, (int)ps.size(), ps.data(), &q, nullptr));
                for (size_t i = 0; i < ps.size(); ++i)
                    CHECK(read_out(fs[idx[i]], ps[i].u, ps[i].v, rs[idx[i]]) == ref[idx[i]],
                          "batched %s pair %d (beta %g, round %d) differs from its plain solve",
                          scheme == FLOW_PDR ? "pDR" : "ALG1", idx[i], beta, round);
                for (float* b : bufs) hipFree(b);
            }
            // served: submit, step and poll in a random order; every result equals the plain solve
            flow_server* srv = nullptr;
            OK(flow_server_create(ctx, &p, (size_t)64 << 20, 1 + (int)(rng() % 3), nullptr, &srv));
            std::vector<uint64_t> tk(fs.size());
            std::vector<flow_result> rs(fs.size());
            std::vector<float*> us(fs.size()), vs(fs.size());
            for (size_t k = 0; k < fs.size(); ++k) {
                hipMalloc(&us[k], sizeof(float) * fs[k].H * fs[k].W);
                hipMalloc(&vs[k], sizeof(float) * fs[k].H * fs[k].W);
                flow_pair q{fs[k].I0, fs[k].I1, fs[k].H, fs[k].W, fs[k].W, us[k], vs[k], fs[k].W, &rs[k], fs[k].levels};
                OK(flow_server_submit(srv, &q, &tk[k]));
                for (int st = (int)(rng() % 3); st > 0; --st) OK(flow_server_step(srv, nullptr, nullptr));
            }
            OK(flow_server_drain(srv));
            for (size_t k = 0; k < fs.size(); ++k) {
                int32_t done = 0;
                OK(flow_server_poll(srv, tk[k], &done));
                CHECK(done == 1 && read_out(fs[k], us[k], vs[k], rs[k]) == ref[k],
                      "served %s pair %zu (beta %g) differs from its plain solve", scheme == FLOW_PDR ? "pDR" : "ALG1",
                      k, beta);
                hipFree(us[k]);
                hipFree(vs[k]);
            }
            OK(flow_server_destroy(srv));
        }
    for (auto& f : fs) {
        hipFree(f.I0);
        hipFree(f.I1);
    }
    flow_destroy(ctx);
}

int main(int argc, char** argv) {
    const unsigned seed = argc > 1 ? (unsigned)std::strtoul(argv[1], nullptr, 10) : 1u;
    std::mt19937 rng(seed);
    test_range_alloc(rng);
    std::printf("range allocator: %d failed checks\n", g_fail);
    test_planners(rng);
    std::printf("planners: %d failed checks\n", g_fail);
    test_solves(rng);
    std::printf("solves: %d failed checks (%ld toy launches)\n", g_fail, fake_device_launches());
    test_pd_solves(rng);
    std::printf("pDR / ALG1 solves: %d failed checks (%ld toy launches)\n", g_fail, fake_device_launches());
    test_pd_batches(rng);
    std::printf("pDR / ALG1 batches: %d failed checks (%ld toy launches)\n", g_fail, fake_device_launches());
    if (g_fail) {
        std::printf("FAILED (%d checks)\n", g_fail);
        return 1;
    }
    std::printf("HOST LOGIC OK\n");
    return 0;
}
