// Scheduling core of the serving runtime: admission, batching and retirement
// of cube tiles, written against an abstract executor so that it builds and
// runs without a GPU (the HIP executor lives in serve.hip; a stub executor
// drives the same code in the host tests).
//
// Life of a tile:
//   submit     -- the caller's measurements are copied into the pinned host
//                 staging pool when they fit there now, otherwise into
//                 pageable memory (never waits);
//   pending    -- tiles leave the arrival queue strictly in order when their
//                 device block (Y in; X, support, stats out) fits in the
//                 device pool; their input copy is then enqueued and its
//                 host staging is freed as soon as that copy has completed;
//   admitted   -- the tile is cut into chunks of at most chunk_pixels; a
//                 batch takes chunks of any admitted tiles (any dictionary,
//                 any band count) up to batch_pixels and max_items and is
//                 enqueued as one or more launches (one per parameter class)
//                 that wait on the device for the input copies of their
//                 tiles; at most max_inflight batches are in flight, so tiles
//                 admitted while a batch runs join the next one;
//   computed   -- once all its chunks are done, the results are copied into
//                 a host result block taken from the pinned pool when it
//                 fits there now, otherwise into pageable memory (never
//                 waits); when that copy has completed, the device block is
//                 freed and the tile is finished;
//   polled     -- the caller reads the host results until it releases the
//                 tag.
// Nothing in this cycle waits on host memory: the only resource admission
// waits for is the device pool, and device blocks are freed by the result
// copies, which never wait.  So every submitted tile finishes whatever the
// caller does with its polled results.
//
// Threading: one scheduler thread runs step() under the lock; submit, poll,
// release, drain and stats may be called from any thread.  Every executor
// call is made under the lock and must not block on device work, except
// copies into pageable memory, which the executor may complete before
// returning.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <vector>

#include "../../include/csrec.h"

namespace csrec {
namespace serving {

inline size_t al256(size_t a) { return (a + 255) / 256 * 256; }

// First-fit allocator of byte ranges [0, capacity) in 256-byte granules.
class RangePool {
   public:
    void init(size_t cap) {
        free_.clear();
        used_.clear();
        if (cap) free_[0] = cap;
        cap_ = cap;
        in_use_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = al256(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t o = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[o + bytes] = len - bytes;
                used_[o] = bytes;
                in_use_ += bytes;
                *off = o;
                return true;
            }
        }
        return false;
    }
    void release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second, start = off;
        in_use_ -= len;
        used_.erase(u);
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + len) {
            len += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(off);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    size_t capacity() const { return cap_; }
    size_t in_use() const { return in_use_; }

   private:
    size_t cap_ = 0, in_use_ = 0;
    std::map<size_t, size_t> free_, used_;
};

// gOMP parameters of one tile after defaults and checks.  Tiles with equal
// same_launch() share launches; max_iter may differ between them.
struct TileParams {
    int K = 0, S = 0, max_iter = 0, prune = 0, prec = 0;
    float res_tol = 0.f, eps = 0.f;
    double pivot_fallback = 0.0, redo_tol = 0.0;
    bool same_launch(const TileParams& o) const {
        return K == o.K && S == o.S && prune == o.prune && prec == o.prec && res_tol == o.res_tol && eps == o.eps &&
               pivot_fallback == o.pivot_fallback && redo_tol == o.redo_tol;
    }
};

struct Tile {
    uint64_t tag = 0;
    int dict = 0;
    int64_t P = 0;
    int M = 0, N = 0;
    TileParams prm;
    // measurements staged on the host: pinned pool range or pageable copy
    bool hin_pool = false;
    size_t hin_off = 0;
    std::vector<float> hin_vec;
    // device block: Y | X | support | stats
    bool dev_held = false;
    size_t dev_off = 0;
    // host results: pinned pool range or pageable block
    bool hout_pool = false;
    size_t hout_off = 0;
    std::vector<char> hout_vec;
    uint64_t ev_in = 0, ev_out = 0;   // executor handles, 0 = none
    bool in_done = false;
    int64_t issued = 0, done = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = CSREC_OK;

    size_t y_bytes() const { return al256((size_t)P * M * 4); }
    size_t x_bytes() const { return al256((size_t)P * N * 4); }
    size_t s_bytes() const { return al256((size_t)P * prm.K * 4); }
    size_t st_bytes() const { return al256((size_t)P * sizeof(csrec_pixel_stats)); }
    size_t dev_bytes() const { return y_bytes() + x_bytes() + s_bytes() + st_bytes(); }
    size_t out_bytes() const { return x_bytes() + s_bytes() + st_bytes(); }
    // offsets inside the device block and inside the host result block
    size_t dev_x() const { return y_bytes(); }
    size_t dev_s() const { return y_bytes() + x_bytes(); }
    size_t dev_st() const { return y_bytes() + x_bytes() + s_bytes(); }
    size_t out_s() const { return x_bytes(); }
    size_t out_st() const { return x_bytes() + s_bytes(); }
};

// A piece of one tile in a batch: pixels [p0, p0 + np).
struct Chunk {
    Tile* tile;
    int64_t p0, np;
};

// The device side.  Every start call enqueues asynchronous work and returns
// a handle; query() reports 0 (done), 1 (pending) or a negative CSREC_E_*
// code; forget() releases a handle.  The calls are made under the
// scheduler's lock.
class Executor {
   public:
    virtual ~Executor() {}
    // copy the tile's staged measurements into Y of its device block
    virtual int input_start(Tile& t, uint64_t* h) = 0;
    // solve the chunks (every chunk's tile has its input copy enqueued);
    // chunks of one parameter class are contiguous
    virtual int launch(const std::vector<Chunk>& chunks, uint64_t* h) = 0;
    // copy X, support and stats of the tile into its host result block
    virtual int output_start(Tile& t, uint64_t* h) = 0;
    virtual int query(uint64_t h) = 0;
    virtual void forget(uint64_t h) = 0;
    // address of a pinned host pool range
    virtual char* host_ptr(size_t off) = 0;
    // waits for every enqueued operation (error and shutdown paths only)
    virtual void wait_idle() = 0;
};

struct Config {
    size_t dev_bytes = 0;        // device pool
    size_t host_bytes = 0;       // pinned host staging pool
    int64_t batch_pixels = 0;    // pixels per batch
    int64_t chunk_pixels = 0;    // largest piece of one tile in a batch
    int max_items = 0;           // chunks per batch
    int max_inflight = 2;        // batches in flight
};

// Counters and time integrals since creation (seconds).
struct Counters {
    int64_t tiles_submitted = 0, tiles_finished = 0, batches = 0, pixels_launched = 0;
    int64_t host_in_pageable = 0, host_out_pageable = 0;
    double busy_s = 0;           // time with at least one batch in flight
    double slot_px_s = 0;        // integral of the pixels in flight
    double pool_bytes_s = 0;     // integral of the device pool bytes in use
    double elapsed_s = 0;
};

class Scheduler {
   public:
    Scheduler(const Config& cfg, Executor* ex) : cfg_(cfg), ex_(ex), t0_(std::chrono::steady_clock::now()) {
        dev_.init(cfg.dev_bytes);
        host_.init(cfg.host_bytes);
        t_last_ = 0;
    }
    ~Scheduler() { shutdown(); }

    void start() { th_ = std::thread([this] { loop(); }); }

    // Stops after every submitted tile has finished; frees what remains.
    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopped_) return;
            stop_ = true;
            cv_.notify_all();
        }
        if (th_.joinable()) th_.join();
        std::lock_guard<std::mutex> lk(mu_);
        ex_->wait_idle();
        for (auto& kv : polled_) drop(kv.second.get());
        for (auto& t : finished_) drop(t.get());
        polled_.clear();
        finished_.clear();
        stopped_ = true;
    }

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
    }

    // Queues a tile.  CSREC_E_INVAL for a tag that is still in flight or
    // polled and not released; CSREC_E_BUDGET when the tile alone exceeds
    // the device pool or the batch limits.
    int submit(int dict, int M, int N, const TileParams& prm, const float* Y, int64_t P, uint64_t tag) {
        std::unique_ptr<Tile> t(new Tile());
        t->t_submit = now();
        t->tag = tag;
        t->dict = dict;
        t->P = P;
        t->M = M;
        t->N = N;
        t->prm = prm;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stop_) return CSREC_E_INVAL;
            if (error_) return error_;
            if (tags_.count(tag)) return CSREC_E_INVAL;
            if (t->dev_bytes() > dev_.capacity()) return CSREC_E_BUDGET;
            if (P > 0) t->hin_pool = host_.alloc((size_t)P * M * 4, &t->hin_off);
            tags_.insert(tag);
        }
        // the copy runs outside the lock: the host range (or vector) is the tile's own
        if (P > 0) {
            if (t->hin_pool) {
                char* dst;
                {
                    std::lock_guard<std::mutex> lk(mu_);
                    dst = ex_->host_ptr(t->hin_off);
                }
                std::memcpy(dst, Y, (size_t)P * M * 4);
            } else {
                t->hin_vec.assign(Y, Y + (size_t)P * M);
            }
        }
        std::lock_guard<std::mutex> lk(mu_);
        ++ctr_.tiles_submitted;
        if (!t->hin_pool && P > 0) ++ctr_.host_in_pageable;
        if (P == 0) {
            t->t_admit = t->t_done = t->t_submit;
            ++ctr_.tiles_finished;
            finished_.push_back(std::move(t));
        } else {
            ++outstanding_;
            pending_.push_back(std::move(t));
        }
        cv_.notify_all();
        return CSREC_OK;
    }

    // Moves up to max finished tiles to the polled set and returns them; the
    // pointers stay valid until release(tag).
    int poll(std::vector<const Tile*>& out, int max) {
        std::lock_guard<std::mutex> lk(mu_);
        int k = 0;
        while (k < max && !finished_.empty()) {
            std::unique_ptr<Tile> t = std::move(finished_.front());
            finished_.pop_front();
            out.push_back(t.get());
            polled_[t->tag] = std::move(t);
            ++k;
        }
        return k;
    }

    // Pointer to a tile's host results (X, then support and stats at
    // out_s() / out_st()), or null when it has none.
    char* results(const Tile* t) {
        if (t->hout_pool) return ex_->host_ptr(t->hout_off);
        return t->hout_vec.empty() ? nullptr : const_cast<char*>(t->hout_vec.data());
    }

    int release(uint64_t tag) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = polled_.find(tag);
        if (it == polled_.end()) return CSREC_OK;
        drop(it->second.get());
        polled_.erase(it);
        tags_.erase(tag);
        return CSREC_OK;
    }

    int drain() {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [this] { return outstanding_ == 0; });
        return error_;
    }

    Counters counters() {
        std::lock_guard<std::mutex> lk(mu_);
        account(now());
        return ctr_;
    }

    // test hooks
    size_t dev_in_use() {
        std::lock_guard<std::mutex> lk(mu_);
        return dev_.in_use();
    }
    size_t host_in_use() {
        std::lock_guard<std::mutex> lk(mu_);
        return host_.in_use();
    }

   private:
    void account(double t) {
        const double dt = t - t_last_;
        if (dt > 0) {
            if (!inflight_.empty()) ctr_.busy_s += dt;
            ctr_.slot_px_s += dt * (double)px_inflight_;
            ctr_.pool_bytes_s += dt * (double)dev_.in_use();
            t_last_ = t;
        }
        ctr_.elapsed_s = t;
    }

    void fail(int code) {
        if (!error_) error_ = code;
    }

    void drop(Tile* t) {
        if (t->dev_held) dev_.release(t->dev_off);
        if (t->hin_pool) host_.release(t->hin_off);
        if (t->hout_pool) host_.release(t->hout_off);
        if (t->ev_in) ex_->forget(t->ev_in);
        if (t->ev_out) ex_->forget(t->ev_out);
        t->dev_held = t->hin_pool = t->hout_pool = false;
        t->ev_in = t->ev_out = 0;
        std::vector<float>().swap(t->hin_vec);
    }

    void finish(std::unique_ptr<Tile> t, int status) {
        if (status != CSREC_OK) t->status = status;
        t->t_done = now();
        if (t->dev_held) dev_.release(t->dev_off);
        t->dev_held = false;
        if (t->hin_pool) host_.release(t->hin_off);
        t->hin_pool = false;
        std::vector<float>().swap(t->hin_vec);
        --outstanding_;
        ++ctr_.tiles_finished;
        finished_.push_back(std::move(t));
    }

    // One pass over the state machine; true when anything changed.
    bool step() {
        bool worked = false;
        account(now());
        // ---- retire batches in order
        while (!inflight_.empty()) {
            Batch& b = inflight_.front();
            const int q = ex_->query(b.ev);
            if (q == 1) break;
            if (q < 0) fail(q);
            for (auto& c : b.chunks) c.tile->done += c.np;
            px_inflight_ -= b.pixels;
            ex_->forget(b.ev);
            inflight_.pop_front();
            worked = true;
        }
        // ---- input copies that completed free their host staging
        for (auto& t : admitted_) {
            if (t->in_done || !t->ev_in) continue;
            const int q = ex_->query(t->ev_in);
            if (q == 1) continue;
            if (q < 0) fail(q);
            t->in_done = true;
            ex_->forget(t->ev_in);
            t->ev_in = 0;
            if (t->hin_pool) host_.release(t->hin_off);
            t->hin_pool = false;
            std::vector<float>().swap(t->hin_vec);
            worked = true;
        }
        // ---- solved tiles: result copy into pinned memory, else pageable
        for (auto it = admitted_.begin(); it != admitted_.end();) {
            Tile* t = it->get();
            if (t->done < t->P || !t->in_done) {
                ++it;
                continue;
            }
            t->hout_pool = host_.alloc(t->out_bytes(), &t->hout_off);
            if (!t->hout_pool) {
                t->hout_vec.assign(t->out_bytes(), 0);
                ++ctr_.host_out_pageable;
            }
            const int e = ex_->output_start(*t, &t->ev_out);
            if (e) fail(e);
            copying_.push_back(std::move(*it));
            it = admitted_.erase(it);
            worked = true;
        }
        // ---- result copies that completed
        for (auto it = copying_.begin(); it != copying_.end();) {
            Tile* t = it->get();
            const int q = t->ev_out ? ex_->query(t->ev_out) : 0;
            if (q == 1) {
                ++it;
                continue;
            }
            if (q < 0) fail(q);
            if (t->ev_out) ex_->forget(t->ev_out);
            t->ev_out = 0;
            std::unique_ptr<Tile> own = std::move(*it);
            it = copying_.erase(it);
            finish(std::move(own), q < 0 ? q : CSREC_OK);
            worked = true;
        }
        if (error_) return worked;
        // ---- admission in arrival order
        while (!pending_.empty()) {
            Tile* t = pending_.front().get();
            if (!dev_.alloc(t->dev_bytes(), &t->dev_off)) break;
            t->dev_held = true;
            t->t_admit = now();
            const int e = ex_->input_start(*t, &t->ev_in);
            if (e) fail(e);
            admitted_.push_back(std::move(pending_.front()));
            pending_.pop_front();
            worked = true;
            if (e) return worked;
        }
        // ---- issue a batch: chunks in admission order, grouped by parameter class
        if ((int)inflight_.size() < cfg_.max_inflight) {
            std::vector<Chunk> chunks;
            int64_t room = cfg_.batch_pixels;
            std::vector<Tile*> order;
            for (auto& up : admitted_)
                if (up->issued < up->P) order.push_back(up.get());
            std::vector<bool> taken(order.size(), false);
            for (size_t lead = 0; lead < order.size() && room > 0 && (int)chunks.size() < cfg_.max_items; ++lead) {
                if (taken[lead]) continue;
                const TileParams cls = order[lead]->prm;
                for (size_t i = lead; i < order.size(); ++i) {
                    Tile* t = order[i];
                    if (taken[i] || !t->prm.same_launch(cls)) continue;
                    taken[i] = true;
                    while (t->issued < t->P && room > 0 && (int)chunks.size() < cfg_.max_items) {
                        const int64_t np = std::min({t->P - t->issued, cfg_.chunk_pixels, room});
                        chunks.push_back(Chunk{t, t->issued, np});
                        t->issued += np;
                        room -= np;
                    }
                    if (room <= 0 || (int)chunks.size() >= cfg_.max_items) break;
                }
            }
            if (!chunks.empty()) {
                Batch b;
                b.chunks = chunks;
                b.pixels = cfg_.batch_pixels - room;
                const int e = ex_->launch(chunks, &b.ev);
                if (e) fail(e);
                px_inflight_ += b.pixels;
                ++ctr_.batches;
                ctr_.pixels_launched += b.pixels;
                inflight_.push_back(std::move(b));
                worked = true;
            }
        }
        return worked;
    }

    // After an error: wait for the device, then fail every unfinished tile.
    void fail_all() {
        ex_->wait_idle();
        for (auto& b : inflight_) {
            ex_->forget(b.ev);
            px_inflight_ -= b.pixels;
        }
        inflight_.clear();
        for (auto* lst : {&admitted_, &copying_}) {
            for (auto& t : *lst) {
                if (t->ev_in) ex_->forget(t->ev_in);
                if (t->ev_out) ex_->forget(t->ev_out);
                t->ev_in = t->ev_out = 0;
                finish(std::move(t), error_);
            }
            lst->clear();
        }
        for (auto& t : pending_) finish(std::move(t), error_);
        pending_.clear();
    }

    // Timed wait on the condition variable against the system clock (a wait
    // on the steady clock goes through pthread_cond_clockwait, which some
    // thread sanitizers do not see release the mutex).
    template <class D>
    void nap(std::unique_lock<std::mutex>& lk, D d) {
        cv_.wait_until(lk, std::chrono::system_clock::now() + d);
    }

    void loop() {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            if (error_) {
                fail_all();
                cv_.notify_all();
                if (stop_) break;
                nap(lk, std::chrono::milliseconds(1));
                continue;
            }
            if (stop_ && pending_.empty() && admitted_.empty() && copying_.empty() && inflight_.empty()) break;
            const bool worked = step();
            if (worked) cv_.notify_all();
            if (!worked) nap(lk, std::chrono::microseconds(50));
        }
        account(now());
        cv_.notify_all();
    }

    struct Batch {
        uint64_t ev = 0;
        std::vector<Chunk> chunks;
        int64_t pixels = 0;
    };

    Config cfg_;
    Executor* ex_;
    std::chrono::steady_clock::time_point t0_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::thread th_;
    bool stop_ = false, stopped_ = false;
    int error_ = CSREC_OK;
    int64_t outstanding_ = 0;
    RangePool dev_, host_;
    std::unordered_set<uint64_t> tags_;
    std::deque<std::unique_ptr<Tile>> pending_;
    std::deque<std::unique_ptr<Tile>> admitted_;
    std::deque<std::unique_ptr<Tile>> copying_;
    std::deque<std::unique_ptr<Tile>> finished_;
    std::map<uint64_t, std::unique_ptr<Tile>> polled_;
    std::deque<Batch> inflight_;
    int64_t px_inflight_ = 0;
    double t_last_ = 0;
    Counters ctr_;
};

}  // namespace serving
}  // namespace csrec
