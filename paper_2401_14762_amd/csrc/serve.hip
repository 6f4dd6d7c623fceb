// Serving runtime: continuous batching of cube tiles through gOMP (Alg. 3).
//
// Host side of the request loop.  One scheduler thread per server:
//   admission  -- tiles leave the arrival queue in order when their device
//                 buffers (Y in, X / support / stats out) fit in the pool;
//   batching   -- admitted tiles are cut into pixel chunks; one batch takes
//                 chunks of several tiles (any band counts) up to the batch
//                 capacity and runs them in grouped launches, at most two
//                 batches in flight on the compute stream, so tiles admitted
//                 while a batch runs join the next one;
//   retirement -- a finished batch credits its chunks; a tile whose pixels
//                 are all done is copied back on the copy stream, its pool
//                 space freed and its latency stamped.
// Dictionaries (A and its Gram matrix in FP32 and FP64) stay on the device
// from csrec_server_add_dict until destroy; the per-pixel solver state of a
// batch lives in the batch workspace.  Nothing is allocated on the device
// after creation except dictionaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "common.hpp"

namespace csrec {
namespace {

double now_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// First-fit allocator over one device buffer (256-byte granules).
class Pool {
   public:
    void init(char* base, size_t bytes) {
        base_ = base;
        free_.clear();
        free_[0] = bytes;
        cap_ = bytes;
    }
    char* alloc(size_t bytes) {
        bytes = align_up(bytes, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_[off] = bytes;
                return base_ + off;
            }
        }
        return nullptr;
    }
    void release(char* p) {
        const size_t off = (size_t)(p - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second;
        used_.erase(u);
        size_t start = off;
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

   private:
    char* base_ = nullptr;
    size_t cap_ = 0;
    std::map<size_t, size_t> free_, used_;
};

struct Dict {
    int M = 0, N = 0, imax = 0;
    float* A = nullptr;
    float* AT = nullptr;
    float* G32 = nullptr;
    double* G64 = nullptr;
};

struct Tile {
    uint64_t tag = 0;
    int dict = 0;
    int64_t P = 0;
    std::vector<float> Yh;                 // host copy of the measurements until admitted
    char* mem = nullptr;                   // pool allocation
    float* dY = nullptr;
    float* dX = nullptr;
    int32_t* dS = nullptr;
    csrec_pixel_stats* dSt = nullptr;
    int64_t issued = 0, done = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = CSREC_OK;
    std::vector<float> X;
    std::vector<int32_t> S;
    std::vector<csrec_pixel_stats> St;
};

struct Batch {
    hipEvent_t ev = nullptr;
    std::vector<std::pair<Tile*, int64_t>> parts;
};

size_t tile_bytes(const Dict& d, int64_t P, int K) {
    return align_up((size_t)P * d.M * 4, 256) + align_up((size_t)P * d.N * 4, 256) +
           align_up((size_t)P * K * 4, 256) + align_up((size_t)P * sizeof(csrec_pixel_stats), 256);
}

}  // namespace
}  // namespace csrec

struct csrec_server {
    csrec_server_cfg cfg{};
    std::chrono::steady_clock::time_point t0;
    hipStream_t compute = nullptr, copy = nullptr;
    char* pool_mem = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    void* table_dev = nullptr;
    void* table_host[2] = {nullptr, nullptr};
    int table_flip = 0;
    int max_items = 0;
    csrec::Pool pool;
    std::vector<csrec::Dict> dicts;
    csrec::GreedyLaunch proto{};          // maximal shape of the batch workspace layout
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<csrec::Tile>> pending;
    std::vector<std::unique_ptr<csrec::Tile>> admitted;
    std::deque<std::unique_ptr<csrec::Tile>> finished;   // not yet polled
    std::map<uint64_t, std::unique_ptr<csrec::Tile>> polled;
    std::deque<csrec::Batch> inflight;
    std::thread th;
    bool stop = false;
    int error = CSREC_OK;
    int64_t outstanding = 0;
};

namespace csrec {
namespace {

// One scheduler step under the lock; returns true when it did something.
bool schedule_once(csrec_server* s) {
    bool worked = false;
    // ---- retire finished batches (oldest first)
    while (!s->inflight.empty()) {
        Batch& b = s->inflight.front();
        const hipError_t q = hipEventQuery(b.ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
            set_hip_error(q);
            s->error = CSREC_E_DEVICE;
        }
        for (auto& pr : b.parts) {
            Tile* t = pr.first;
            t->done += pr.second;
            if (t->done == t->P) {
                const int K = s->cfg.gomp.K;
                const Dict& d = s->dicts[t->dict];
                t->X.resize((size_t)t->P * d.N);
                t->S.resize((size_t)t->P * K);
                t->St.resize((size_t)t->P);
                hipError_t e = hipStreamWaitEvent(s->copy, b.ev, 0);
                if (e == hipSuccess) e = hipMemcpyAsync(t->X.data(), t->dX, t->X.size() * 4, hipMemcpyDeviceToHost, s->copy);
                if (e == hipSuccess) e = hipMemcpyAsync(t->S.data(), t->dS, t->S.size() * 4, hipMemcpyDeviceToHost, s->copy);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(t->St.data(), t->dSt, t->St.size() * sizeof(csrec_pixel_stats),
                                       hipMemcpyDeviceToHost, s->copy);
                if (e == hipSuccess) e = hipStreamSynchronize(s->copy);
                if (e != hipSuccess) {
                    set_hip_error(e);
                    t->status = CSREC_E_DEVICE;
                }
                t->t_done = now_since(s->t0);
                s->pool.release(t->mem);
                t->mem = nullptr;
                std::vector<float>().swap(t->Yh);
                for (auto it = s->admitted.begin(); it != s->admitted.end(); ++it)
                    if (it->get() == t) {
                        s->finished.push_back(std::move(*it));
                        s->admitted.erase(it);
                        break;
                    }
                --s->outstanding;
            }
        }
        hipEventDestroy(b.ev);
        s->inflight.pop_front();
        worked = true;
    }
    // ---- admission in arrival order
    while (!s->pending.empty()) {
        Tile* t = s->pending.front().get();
        const Dict& d = s->dicts[t->dict];
        const size_t need = tile_bytes(d, t->P, s->cfg.gomp.K);
        char* m = s->pool.alloc(need);
        if (!m) break;
        t->mem = m;
        t->dY = reinterpret_cast<float*>(m);
        t->dX = reinterpret_cast<float*>(m + align_up((size_t)t->P * d.M * 4, 256));
        t->dS = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(t->dX) + align_up((size_t)t->P * d.N * 4, 256));
        t->dSt = reinterpret_cast<csrec_pixel_stats*>(reinterpret_cast<char*>(t->dS) +
                                                      align_up((size_t)t->P * s->cfg.gomp.K * 4, 256));
        const hipError_t e = hipMemcpyAsync(t->dY, t->Yh.data(), t->Yh.size() * 4, hipMemcpyHostToDevice, s->compute);
        if (e != hipSuccess) {
            set_hip_error(e);
            s->error = CSREC_E_DEVICE;
        }
        t->t_admit = now_since(s->t0);
        s->admitted.push_back(std::move(s->pending.front()));
        s->pending.pop_front();
        worked = true;
    }
    // ---- issue a batch
    if (s->inflight.size() < 2) {
        std::vector<GreedyTileItem> items;
        Batch b;
        int64_t room = s->cfg.batch_pixels;
        for (auto& up : s->admitted) {
            Tile* t = up.get();
            while (t->issued < t->P && room > 0 && (int)items.size() < s->max_items) {
                const int64_t np = std::min({t->P - t->issued, s->cfg.chunk_pixels, room});
                const Dict& d = s->dicts[t->dict];
                GreedyTileItem it{};
                it.A = d.A;
                it.dict = d.AT;
                it.Y = t->dY;
                it.X = t->dX;
                it.support = t->dS;
                it.stats = t->dSt;
                it.G32 = d.G32;
                it.G64 = d.G64;
                it.M = d.M;
                it.N = d.N;
                it.max_iter = d.imax;
                it.p0 = t->issued;
                it.np = np;
                items.push_back(it);
                b.parts.push_back({t, np});
                t->issued += np;
                room -= np;
            }
            if (room <= 0 || (int)items.size() >= s->max_items) break;
        }
        if (!items.empty()) {
            int e = greedy_group_launch(s->proto, items.data(), (int)items.size(), s->cfg.batch_pixels, s->ws,
                                        s->table_host[s->table_flip], s->table_dev, s->compute);
            s->table_flip ^= 1;
            hipError_t he = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
            if (he == hipSuccess) he = hipEventRecord(b.ev, s->compute);
            if (e != CSREC_OK || he != hipSuccess) {
                if (he != hipSuccess) set_hip_error(he);
                s->error = e != CSREC_OK ? e : CSREC_E_DEVICE;
            }
            s->inflight.push_back(std::move(b));
            worked = true;
        }
    }
    return worked;
}

void scheduler(csrec_server* s) {
    hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        if (s->stop && s->pending.empty() && s->admitted.empty() && s->inflight.empty()) break;
        if (s->error != CSREC_OK && s->inflight.empty()) {
            // fail every queued tile and stop issuing work
            for (auto& t : s->pending) {
                t->status = s->error;
                --s->outstanding;
                s->finished.push_back(std::move(t));
            }
            s->pending.clear();
            for (auto& t : s->admitted) {
                t->status = s->error;
                if (t->mem) s->pool.release(t->mem);
                --s->outstanding;
                s->finished.push_back(std::move(t));
            }
            s->admitted.clear();
            s->cv.notify_all();
            if (s->stop) break;
            s->cv.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        const bool worked = schedule_once(s);
        if (worked) s->cv.notify_all();
        if (!worked) s->cv.wait_for(lk, std::chrono::microseconds(50));
    }
    s->cv.notify_all();
}

}  // namespace
}  // namespace csrec

using namespace csrec;

extern "C" {

int32_t csrec_server_create(const csrec_server_cfg* cfg, csrec_server** out) {
    if (!cfg || !out || cfg->struct_size != (int32_t)sizeof(csrec_server_cfg)) return CSREC_E_INVAL;
    const csrec_gomp_params& g = cfg->gomp;
    if (g.struct_size != (int32_t)sizeof(csrec_gomp_params) || g.K < 1 || g.S < 1 || g.S > 8 || g.max_iter < 0 ||
        g.prec != CSREC_PREC_F32 || (g.prune != CSREC_PRUNE_EACH && g.prune != CSREC_PRUNE_FINAL) ||
        !(g.res_tol >= 0) || !(g.eps >= 0) || !(g.pivot_fallback >= 0))
        return g.prec != CSREC_PREC_F32 ? CSREC_E_UNSUPPORTED : CSREC_E_INVAL;
    if (cfg->hbm_budget_bytes < 4096 || cfg->batch_pixels < 256 || cfg->chunk_pixels < 1) return CSREC_E_INVAL;
    std::unique_ptr<csrec_server> s(new csrec_server());
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    CSREC_HIP_TRY(hipSetDevice(cfg->device));
    // the batch workspace is laid out for the largest shape a dictionary may have
    GreedyLaunch& p = s->proto;
    p.kind = GREEDY_GOMP;
    p.M = 96;
    p.N = CSREC_MAX_N;
    p.K = g.K;
    p.S = g.S;
    p.max_iter = g.max_iter > 0 ? g.max_iter : std::min(g.K, 96 / g.S);
    if (g.S * p.max_iter > GREEDY_CMAX || g.K > GREEDY_CMAX) return CSREC_E_SHAPE;
    p.prune = g.prune;
    p.prec = g.prec;
    p.res_tol = (float)g.res_tol;
    p.eps = (float)g.eps;
    p.pivot_fallback = g.pivot_fallback;
    s->ws_bytes = greedy_group_workspace(p, cfg->batch_pixels);
    s->max_items = (int)std::min<int64_t>(4096, cfg->batch_pixels);
    CSREC_HIP_TRY(hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking));
    CSREC_HIP_TRY(hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking));
    CSREC_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&s->pool_mem), cfg->hbm_budget_bytes));
    CSREC_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&s->ws), s->ws_bytes));
    const size_t tb = align_up((size_t)s->max_items * greedy_group_item_bytes(), 256) +
                      (size_t)s->max_items * gomp_coop_item_bytes();
    CSREC_HIP_TRY(hipMalloc(&s->table_dev, tb));
    CSREC_HIP_TRY(hipHostMalloc(&s->table_host[0], tb, hipHostMallocDefault));
    CSREC_HIP_TRY(hipHostMalloc(&s->table_host[1], tb, hipHostMallocDefault));
    s->pool.init(s->pool_mem, cfg->hbm_budget_bytes);
    csrec_server* raw = s.release();
    raw->th = std::thread(scheduler, raw);
    *out = raw;
    return CSREC_OK;
}

int32_t csrec_server_add_dict(csrec_server* s, const float* A_host, int32_t M, int32_t N, int32_t* dict_id) {
    if (!s || !A_host || !dict_id) return CSREC_E_INVAL;
    if (M < 1 || M >= N || N > CSREC_MAX_N) return CSREC_E_SHAPE;
    if (M > 96) return CSREC_E_UNSUPPORTED;
    const csrec_gomp_params& g = s->cfg.gomp;
    Dict d;
    d.M = M;
    d.N = N;
    d.imax = g.max_iter > 0 ? g.max_iter : std::min(g.K, M / g.S);
    if (d.imax < 1 || g.S * d.imax > M || d.imax > s->proto.max_iter) return CSREC_E_SHAPE;
    if (gomp_coop_supported(M, N, g.K, g.S, d.imax) != CSREC_OK) return CSREC_E_UNSUPPORTED;
    CSREC_HIP_TRY(hipSetDevice(s->cfg.device));
    CSREC_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&d.A), (size_t)M * N * 4));
    CSREC_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&d.G32), (size_t)N * N * 4));
    CSREC_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&d.AT), gomp_coop_dict_floats(M, N) * 4));
    if (g.pivot_fallback > 0) CSREC_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&d.G64), (size_t)N * N * 8));
    hipStream_t st = nullptr;
    CSREC_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipError_t e = hipMemcpyAsync(d.A, A_host, (size_t)M * N * 4, hipMemcpyHostToDevice, st);
    int rc = (e == hipSuccess) ? greedy_gram(d.A, M, N, d.G32, d.G64, st) : CSREC_E_DEVICE;
    if (rc == CSREC_OK) gomp_coop_prepare(d.A, M, N, d.AT, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipStreamDestroy(st);
    if (e != hipSuccess) {
        set_hip_error(e);
        return CSREC_E_DEVICE;
    }
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    s->dicts.push_back(d);
    *dict_id = (int32_t)s->dicts.size() - 1;
    return CSREC_OK;
}

int32_t csrec_server_submit(csrec_server* s, int32_t dict_id, const float* Y_host, int64_t P, uint64_t tag) {
    if (!s || (P > 0 && !Y_host) || P < 0) return CSREC_E_INVAL;
    std::unique_ptr<Tile> t(new Tile());
    t->t_submit = now_since(s->t0);
    int M = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (dict_id < 0 || dict_id >= (int32_t)s->dicts.size()) return CSREC_E_INVAL;
        if (s->error) return s->error;
        const Dict& d = s->dicts[dict_id];
        if (tile_bytes(d, P, s->cfg.gomp.K) > s->pool.capacity()) return CSREC_E_BUDGET;
        if (P > s->cfg.batch_pixels * 4096) return CSREC_E_BUDGET;
        M = d.M;
    }
    t->Yh.assign(Y_host, Y_host + (size_t)P * M);   // copied outside the lock
    t->tag = tag;
    t->dict = dict_id;
    t->P = P;
    std::lock_guard<std::mutex> lk(s->mu);
    if (P == 0) {
        t->t_admit = t->t_done = t->t_submit;
        s->finished.push_back(std::move(t));
    } else {
        ++s->outstanding;
        s->pending.push_back(std::move(t));
    }
    s->cv.notify_all();
    return CSREC_OK;
}

int32_t csrec_server_poll(csrec_server* s, csrec_result* out, int32_t max, int32_t* n) {
    if (!s || !n || (max > 0 && !out)) return CSREC_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t k = 0;
    while (k < max && !s->finished.empty()) {
        std::unique_ptr<Tile> t = std::move(s->finished.front());
        s->finished.pop_front();
        const Dict& d = s->dicts[t->dict];
        csrec_result& r = out[k++];
        r.tag = t->tag;
        r.status = t->status;
        r.dict_id = t->dict;
        r.P = t->P;
        r.N = d.N;
        r.K = s->cfg.gomp.K;
        r.X = t->X.data();
        r.support = t->S.data();
        r.stats = t->St.data();
        r.t_submit = t->t_submit;
        r.t_admit = t->t_admit;
        r.t_done = t->t_done;
        s->polled[t->tag] = std::move(t);
    }
    *n = k;
    return CSREC_OK;
}

int32_t csrec_server_release(csrec_server* s, uint64_t tag) {
    if (!s) return CSREC_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->polled.erase(tag);
    return CSREC_OK;
}

int32_t csrec_server_drain(csrec_server* s) {
    if (!s) return CSREC_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [s] { return s->outstanding == 0; });
    return s->error;
}

int32_t csrec_server_destroy(csrec_server* s) {
    if (!s) return CSREC_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    hipSetDevice(s->cfg.device);
    hipStreamSynchronize(s->compute);
    for (auto& d : s->dicts) {
        hipFree(d.A);
        hipFree(d.AT);
        hipFree(d.G32);
        if (d.G64) hipFree(d.G64);
    }
    hipFree(s->pool_mem);
    hipFree(s->ws);
    hipFree(s->table_dev);
    hipHostFree(s->table_host[0]);
    hipHostFree(s->table_host[1]);
    hipStreamDestroy(s->compute);
    hipStreamDestroy(s->copy);
    delete s;
    return CSREC_OK;
}

}  // extern "C"
