// Host test of the serving scheduler (serve_policy.hpp) against a stub
// executor: three worker threads stand in for the device's copy-in, compute
// and copy-out streams, run their operations in order after random delays,
// and compute a known function of each pixel's measurements.  Built with g++
// alone (no HIP), plain and under ThreadSanitizer and AddressSanitizer.
//
// Scenarios: mixed tiles from two submitting threads with a poller that
// keeps results unreleased while a small pinned pool fills (the progress
// guarantee); a burst larger than both pools before any poll; tag reuse;
// budget refusal; per-tile parameter classes kept contiguous in launches;
// an injected device error; shutdown with tiles outstanding.
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2401_14762_amd/csrc/serve_policy.hpp"

using namespace csrec::serving;

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
            std::abort();                                                   \
        }                                                                   \
    } while (0)

// Result of the stub solve for pixel p of a tile: a function of the pixel's
// measurements, the dictionary and the tile's res_tol.
static float expect_x(const float* y, int M, int dict, float res_tol, int n) {
    return y[n % M] * 2.f + (float)dict * 1000.f + (float)n + res_tol;
}

class StubExecutor : public Executor {
   public:
    struct Op {
        std::function<void()> body;
        std::vector<std::shared_ptr<Op>> after;   // must be done before body runs
        std::atomic<int> done{0};
        bool fail = false;
    };

    StubExecutor(size_t dev_bytes, size_t host_bytes, unsigned seed)
        : dev_(dev_bytes), host_(host_bytes), rng_(seed) {
        for (int s = 0; s < 3; ++s) workers_[s] = std::thread([this, s] { run(s); });
    }
    ~StubExecutor() override {
        {
            std::lock_guard<std::mutex> lk(mu_);
            quit_ = true;
        }
        cv_.notify_all();
        for (auto& w : workers_) w.join();
    }

    std::vector<std::pair<int, int>> dims;   // (M, N) per dictionary
    int fail_launch_at = -1;                  // launch index that reports a device error
    std::atomic<int> launches{0};
    std::atomic<int> classes_seen{0};

    int input_start(Tile& t, uint64_t* h) override {
        const char* src = t.hin_pool ? host_.data() + t.hin_off : reinterpret_cast<const char*>(t.hin_vec.data());
        char* dst = dev_.data() + t.dev_off;
        const size_t n = (size_t)t.P * t.M * 4;
        if (!t.hin_pool) {
            // a pageable source is consumed before the call returns
            std::memcpy(dst, src, n);
            return push(0, [] {}, {}, h);
        }
        return push(0, [dst, src, n] { std::memcpy(dst, src, n); }, {}, h);
    }

    int launch(const std::vector<Chunk>& chunks, uint64_t* h) override {
        const int idx = launches.fetch_add(1);
        std::vector<std::shared_ptr<Op>> after;
        // parameter classes are contiguous: a class never reappears later in the batch
        std::vector<TileParams> seen;
        for (size_t i = 0; i < chunks.size(); ++i) {
            const Tile* t = chunks[i].tile;
            if (i == 0 || !t->prm.same_launch(chunks[i - 1].tile->prm)) {
                for (auto& p : seen) CHECK(!p.same_launch(t->prm));
                seen.push_back(t->prm);
            }
            if (!t->in_done && t->ev_in) {
                std::lock_guard<std::mutex> lk(mu_);
                after.push_back(ops_.at(t->ev_in));
            }
            CHECK(chunks[i].np > 0 && chunks[i].p0 + chunks[i].np <= t->P);
        }
        classes_seen.fetch_add((int)seen.size());
        struct Job {
            char* blk;
            int M, N, K, dict;
            float res_tol;
            int64_t p0, np;
            size_t dx, ds, dst;
        };
        std::vector<Job> jobs;
        for (const auto& c : chunks) {
            const Tile* t = c.tile;
            jobs.push_back(Job{dev_.data() + t->dev_off, t->M, t->N, t->prm.K, t->dict, t->prm.res_tol, c.p0, c.np,
                               t->dev_x(), t->dev_s(), t->dev_st()});
        }
        auto body = [jobs] {
            for (const Job& j : jobs) {
                for (int64_t p = j.p0; p < j.p0 + j.np; ++p) {
                    const float* y = reinterpret_cast<const float*>(j.blk) + p * j.M;
                    float* x = reinterpret_cast<float*>(j.blk + j.dx) + p * j.N;
                    int32_t* s = reinterpret_cast<int32_t*>(j.blk + j.ds) + p * j.K;
                    csrec_pixel_stats* st = reinterpret_cast<csrec_pixel_stats*>(j.blk + j.dst) + p;
                    for (int n = 0; n < j.N; ++n) x[n] = expect_x(y, j.M, j.dict, j.res_tol, n);
                    for (int k = 0; k < j.K; ++k) s[k] = (int32_t)((p + k) % j.N);
                    st->iters = (int32_t)(p % 7);
                    st->flags = 0;
                    st->resid = y[0];
                    st->delta = 0.f;
                }
            }
        };
        const int e = push(1, body, after, h);
        if (e == CSREC_OK && idx == fail_launch_at) {
            std::lock_guard<std::mutex> lk(mu_);
            ops_.at(*h)->fail = true;
        }
        return e;
    }

    int output_start(Tile& t, uint64_t* h) override {
        char* dst = t.hout_pool ? host_.data() + t.hout_off : t.hout_vec.data();
        const char* blk = dev_.data() + t.dev_off;
        const size_t nx = (size_t)t.P * t.N * 4, ns = (size_t)t.P * t.prm.K * 4,
                     nst = (size_t)t.P * sizeof(csrec_pixel_stats);
        const size_t ox = t.dev_x(), os = t.dev_s(), ost = t.dev_st(), ds = t.out_s(), dst_ = t.out_st();
        return push(2, [=] {
            std::memcpy(dst, blk + ox, nx);
            std::memcpy(dst + ds, blk + os, ns);
            std::memcpy(dst + dst_, blk + ost, nst);
        }, {}, h);
    }

    int query(uint64_t h) override {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = ops_.find(h);
        CHECK(it != ops_.end());
        if (!it->second->done.load(std::memory_order_acquire)) return 1;
        return it->second->fail ? CSREC_E_DEVICE : 0;
    }

    void forget(uint64_t h) override {
        std::lock_guard<std::mutex> lk(mu_);
        CHECK(ops_.erase(h) == 1);
    }

    char* host_ptr(size_t off) override { return host_.data() + off; }

    void wait_idle() override {
        std::unique_lock<std::mutex> lk(mu_);
        idle_cv_.wait(lk, [this] { return q_[0].empty() && q_[1].empty() && q_[2].empty() && busy_ == 0; });
    }

    size_t live_handles() {
        std::lock_guard<std::mutex> lk(mu_);
        return ops_.size();
    }

   private:
    int push(int stream, std::function<void()> body, std::vector<std::shared_ptr<Op>> after, uint64_t* h) {
        auto op = std::make_shared<Op>();
        op->body = std::move(body);
        op->after = std::move(after);
        {
            std::lock_guard<std::mutex> lk(mu_);
            *h = next_++;
            ops_[*h] = op;
            q_[stream].push_back(op);
        }
        cv_.notify_all();
        return CSREC_OK;
    }

    void run(int s) {
        std::mt19937 rng(1234 + s);
        while (true) {
            std::shared_ptr<Op> op;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return quit_ || !q_[s].empty(); });
                if (q_[s].empty()) return;
                op = q_[s].front();
                q_[s].pop_front();
                ++busy_;
            }
            for (auto& a : op->after)
                while (!a->done.load(std::memory_order_acquire)) std::this_thread::yield();
            std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
            op->body();
            op->done.store(1, std::memory_order_release);
            {
                std::lock_guard<std::mutex> lk(mu_);
                --busy_;
            }
            idle_cv_.notify_all();
        }
    }

    std::vector<char> dev_, host_;
    std::mt19937 rng_;
    std::mutex mu_;
    std::condition_variable cv_, idle_cv_;
    std::deque<std::shared_ptr<Op>> q_[3];
    std::map<uint64_t, std::shared_ptr<Op>> ops_;
    uint64_t next_ = 1;
    int busy_ = 0;
    bool quit_ = false;
    std::thread workers_[3];
};

struct TileIn {
    int dict;
    std::vector<float> Y;
    int64_t P;
    TileParams prm;
};

static TileParams params(float res_tol) {
    TileParams p;
    p.K = 6;
    p.S = 2;
    p.max_iter = 3;
    p.res_tol = res_tol;
    return p;
}

static void verify(Scheduler& sch, const Tile* t, const TileIn& in) {
    CHECK(t->status == CSREC_OK);
    CHECK(t->P == in.P);
    CHECK(t->t_submit <= t->t_admit && t->t_admit <= t->t_done);
    if (t->P == 0) return;
    const char* base = sch.results(t);
    CHECK(base != nullptr);
    const float* X = reinterpret_cast<const float*>(base);
    const int32_t* S = reinterpret_cast<const int32_t*>(base + t->out_s());
    const csrec_pixel_stats* st = reinterpret_cast<const csrec_pixel_stats*>(base + t->out_st());
    for (int64_t p = 0; p < t->P; ++p) {
        const float* y = in.Y.data() + p * t->M;
        for (int n = 0; n < t->N; ++n) CHECK(X[p * t->N + n] == expect_x(y, t->M, in.dict, in.prm.res_tol, n));
        for (int k = 0; k < t->prm.K; ++k) CHECK(S[p * t->prm.K + k] == (int32_t)((p + k) % t->N));
        CHECK(st[p].iters == (int32_t)(p % 7));
        CHECK(st[p].resid == y[0]);
    }
}

static std::vector<TileIn> make_tiles(int n, unsigned seed, int nclasses) {
    std::mt19937 rng(seed);
    std::vector<TileIn> out;
    for (int i = 0; i < n; ++i) {
        TileIn t;
        t.dict = (int)(rng() % 3);
        t.P = (int64_t)(rng() % 3000) + (i % 17 == 0 ? 0 : 1);
        if (i % 17 == 0) t.P = 0;
        const int M = t.dict == 0 ? 40 : (t.dict == 1 ? 80 : 90);
        t.Y.resize((size_t)t.P * M);
        for (auto& v : t.Y) v = (float)(rng() % 1000) * 0.25f;
        t.prm = params(nclasses > 1 ? 0.001f * (float)(i % nclasses) : 0.f);
        out.push_back(std::move(t));
    }
    return out;
}

static const int kM[3] = {40, 80, 90}, kN[3] = {100, 200, 224};

// Mixed traffic: two submitters, a poller that keeps up to `hold` results
// unreleased (so the small pinned pool stays full), per-tile parameter classes.
static void scenario_mixed(size_t dev_bytes, size_t host_bytes, int hold, unsigned seed) {
    const int ntiles = 160;
    std::vector<TileIn> tiles = make_tiles(ntiles, seed, 3);
    StubExecutor ex(dev_bytes, host_bytes, seed);
    Config cfg;
    cfg.dev_bytes = dev_bytes;
    cfg.host_bytes = host_bytes;
    cfg.batch_pixels = 4096;
    cfg.chunk_pixels = 1000;
    cfg.max_items = 64;
    {
        Scheduler sch(cfg, &ex);
        sch.start();
        std::atomic<int> submitted{0};
        auto submitter = [&](int parity) {
            for (int i = parity; i < ntiles; i += 2) {
                const TileIn& t = tiles[i];
                CHECK(sch.submit(t.dict, kM[t.dict], kN[t.dict], t.prm, t.Y.data(), t.P, (uint64_t)i) == CSREC_OK);
                submitted.fetch_add(1);
            }
        };
        std::thread s0(submitter, 0), s1(submitter, 1);
        int got = 0;
        std::deque<uint64_t> held;
        std::vector<bool> seen(ntiles, false);
        while (got < ntiles) {
            std::vector<const Tile*> out;
            sch.poll(out, 7);
            for (const Tile* t : out) {
                CHECK(t->tag < (uint64_t)ntiles && !seen[t->tag]);
                seen[t->tag] = true;
                verify(sch, t, tiles[t->tag]);
                held.push_back(t->tag);
                ++got;
            }
            while ((int)held.size() > hold) {
                CHECK(sch.release(held.front()) == CSREC_OK);
                held.pop_front();
            }
            if (out.empty()) std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        s0.join();
        s1.join();
        CHECK(sch.drain() == CSREC_OK);
        const Counters c = sch.counters();
        CHECK(c.tiles_submitted == ntiles && c.tiles_finished == ntiles);
        int64_t px = 0;
        for (auto& t : tiles) px += t.P;
        CHECK(c.pixels_launched == px);
        CHECK(c.busy_s <= c.elapsed_s + 1e-9);
        CHECK(ex.classes_seen.load() >= ex.launches.load());
        for (uint64_t tag : held) CHECK(sch.release(tag) == CSREC_OK);
        CHECK(sch.dev_in_use() == 0);
        CHECK(sch.host_in_use() == 0);
        std::printf("mixed: %d tiles, %lld batches, %lld inputs and %lld results in pageable memory\n", ntiles,
                    (long long)c.batches, (long long)c.host_in_pageable, (long long)c.host_out_pageable);
    }
    CHECK(ex.live_handles() == 0);
}

// A burst larger than the device pool and the pinned pool, submitted before
// any poll, from one thread: everything finishes, admission keeps arrival order.
static void scenario_burst() {
    const int ntiles = 60;
    std::vector<TileIn> tiles = make_tiles(ntiles, 7, 1);
    const size_t dev_bytes = 6u << 20, host_bytes = 1u << 20;
    StubExecutor ex(dev_bytes, host_bytes, 7);
    Config cfg;
    cfg.dev_bytes = dev_bytes;
    cfg.host_bytes = host_bytes;
    cfg.batch_pixels = 2048;
    cfg.chunk_pixels = 512;
    cfg.max_items = 16;
    Scheduler sch(cfg, &ex);
    sch.start();
    for (int i = 0; i < ntiles; ++i) {
        const TileIn& t = tiles[i];
        CHECK(sch.submit(t.dict, kM[t.dict], kN[t.dict], t.prm, t.Y.data(), t.P, (uint64_t)(100 + i)) == CSREC_OK);
    }
    CHECK(sch.drain() == CSREC_OK);
    std::vector<const Tile*> out;
    CHECK(sch.poll(out, 1000) == ntiles);
    double last_admit = -1;
    std::map<uint64_t, const Tile*> by_tag;
    for (const Tile* t : out) by_tag[t->tag] = t;
    for (int i = 0; i < ntiles; ++i) {
        const Tile* t = by_tag.at((uint64_t)(100 + i));
        verify(sch, t, tiles[i]);
        if (t->P > 0) {
            CHECK(t->t_admit >= last_admit);
            last_admit = t->t_admit;
        }
    }
    const Counters c = sch.counters();
    CHECK(c.host_out_pageable > 0);   // the pinned pool could not hold every result
    for (int i = 0; i < ntiles; ++i) CHECK(sch.release((uint64_t)(100 + i)) == CSREC_OK);
    std::printf("burst: %d tiles, %lld results in pageable memory\n", ntiles, (long long)c.host_out_pageable);
}

static void scenario_tags_and_budget() {
    StubExecutor ex(1u << 20, 1u << 20, 3);
    Config cfg;
    cfg.dev_bytes = 1u << 20;
    cfg.host_bytes = 1u << 20;
    cfg.batch_pixels = 1024;
    cfg.chunk_pixels = 256;
    cfg.max_items = 8;
    Scheduler sch(cfg, &ex);
    sch.start();
    std::vector<float> Y(300 * 80, 1.f);
    const TileParams p = params(0.f);
    CHECK(sch.submit(1, 80, 200, p, Y.data(), 300, 5) == CSREC_OK);
    CHECK(sch.submit(1, 80, 200, p, Y.data(), 300, 5) == CSREC_E_INVAL);   // in flight
    CHECK(sch.drain() == CSREC_OK);
    CHECK(sch.submit(1, 80, 200, p, Y.data(), 300, 5) == CSREC_E_INVAL);   // finished, not polled
    std::vector<const Tile*> out;
    CHECK(sch.poll(out, 4) == 1);
    CHECK(sch.submit(1, 80, 200, p, Y.data(), 300, 5) == CSREC_E_INVAL);   // polled, not released
    CHECK(sch.release(5) == CSREC_OK);
    CHECK(sch.submit(1, 80, 200, p, Y.data(), 300, 5) == CSREC_OK);        // released: reusable
    std::vector<float> big((size_t)5000 * 80, 1.f);
    CHECK(sch.submit(1, 80, 200, p, big.data(), 5000, 6) == CSREC_E_BUDGET);
    CHECK(sch.submit(1, 80, 200, p, big.data(), 5000, 7) == CSREC_E_BUDGET);
    CHECK(sch.drain() == CSREC_OK);
    std::printf("tags and budget: ok\n");
}

// An injected device error: drain returns it, every tile finishes with it,
// later submits are refused, shutdown completes.
static void scenario_error() {
    std::vector<TileIn> tiles = make_tiles(40, 11, 2);
    StubExecutor ex(8u << 20, 2u << 20, 11);
    ex.fail_launch_at = 3;
    Config cfg;
    cfg.dev_bytes = 8u << 20;
    cfg.host_bytes = 2u << 20;
    cfg.batch_pixels = 1024;
    cfg.chunk_pixels = 512;
    cfg.max_items = 8;
    Scheduler sch(cfg, &ex);
    sch.start();
    int accepted = 0;
    for (int i = 0; i < 40; ++i) {
        const TileIn& t = tiles[i];
        const int e = sch.submit(t.dict, kM[t.dict], kN[t.dict], t.prm, t.Y.data(), t.P, (uint64_t)i);
        CHECK(e == CSREC_OK || e == CSREC_E_DEVICE);
        accepted += e == CSREC_OK;
    }
    CHECK(sch.drain() == CSREC_E_DEVICE);
    std::vector<const Tile*> out;
    CHECK(sch.poll(out, 100) == accepted);
    int failed = 0;
    for (const Tile* t : out) failed += t->status == CSREC_E_DEVICE;
    CHECK(failed > 0);
    std::vector<float> Y(80, 1.f);
    CHECK(sch.submit(1, 80, 200, params(0.f), Y.data(), 1, 999) == CSREC_E_DEVICE);
    std::printf("error: %d of %d tiles failed\n", failed, accepted);
}

// Shutdown right after submitting: the destructor waits for every tile.
static void scenario_shutdown() {
    std::vector<TileIn> tiles = make_tiles(30, 5, 1);
    StubExecutor ex(16u << 20, 1u << 20, 5);
    Config cfg;
    cfg.dev_bytes = 16u << 20;
    cfg.host_bytes = 1u << 20;
    cfg.batch_pixels = 4096;
    cfg.chunk_pixels = 1024;
    cfg.max_items = 16;
    {
        Scheduler sch(cfg, &ex);
        sch.start();
        for (int i = 0; i < 30; ++i) {
            const TileIn& t = tiles[i];
            CHECK(sch.submit(t.dict, kM[t.dict], kN[t.dict], t.prm, t.Y.data(), t.P, (uint64_t)i) == CSREC_OK);
        }
    }
    CHECK(ex.live_handles() == 0);
    std::printf("shutdown: ok\n");
}

int main() {
    scenario_tags_and_budget();
    scenario_mixed(24u << 20, 2u << 20, 40, 1);    // small pinned pool, results held
    scenario_mixed(64u << 20, 64u << 20, 0, 2);    // everything pinned
    scenario_burst();
    scenario_error();
    scenario_shutdown();
    std::printf("serve policy: all scenarios passed\n");
    return 0;
}
