// Serving runtime: continuous batching of cube tiles through gOMP (Alg. 3).
//
// Host side of the request loop.  One scheduler thread per server:
//   submission -- the caller's measurements are copied into a pinned host
//                 staging pool (first fit; pageable memory only for a tile
//                 that could never fit it), outside the server lock;
//   admission  -- tiles leave the arrival queue in order when their device
//                 buffers (Y in, X / support / stats out) fit in the device
//                 pool; their input copy runs on the host-to-device stream;
//   batching   -- admitted tiles are cut into pixel chunks; one batch takes
//                 chunks of several tiles (any band counts) up to the batch
//                 capacity and runs them in grouped launches, at most two
//                 batches in flight on the compute stream, so tiles admitted
//                 while a batch runs join the next one; a batch waits (on the
//                 device) for the input copies of its tiles;
//   retirement -- a finished batch credits its chunks; a tile whose pixels
//                 are all done is copied into pinned host result memory on
//                 the device-to-host stream, and once that copy's event has
//                 completed its device memory is freed and its latency
//                 stamped.
// Every HIP call the scheduler makes under the lock is asynchronous (event
// queries, copies between pinned and device memory, launches), so submit and
// poll never wait behind a transfer.  Dictionaries (A, its copies for the
// on-chip kernel and its Gram matrix in FP32 and FP64) stay on the device from
// csrec_server_add_dict until destroy; the per-pixel solver state of a batch
// lives in the batch workspace.  Nothing is allocated on the device after
// creation except dictionaries.
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
    char* hin = nullptr;                   // pinned staging of the measurements (host pool) ...
    std::vector<float> Yv;                 // ... or a pageable copy when the pool cannot hold them
    char* mem = nullptr;                   // device pool allocation
    float* dY = nullptr;
    float* dX = nullptr;
    int32_t* dS = nullptr;
    csrec_pixel_stats* dSt = nullptr;
    hipEvent_t ev_in = nullptr;            // input copy done (host-to-device stream)
    hipEvent_t ev_out = nullptr;           // result copy done (device-to-host stream)
    bool in_waited = false;                // the compute stream already waits on ev_in
    int64_t issued = 0, done = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = CSREC_OK;
    char* hout = nullptr;                  // pinned results (host pool), or the vectors below
    std::vector<float> Xv;
    std::vector<int32_t> Sv;
    std::vector<csrec_pixel_stats> Stv;
    float* X = nullptr;
    int32_t* S = nullptr;
    csrec_pixel_stats* St = nullptr;
};

struct Batch {
    hipEvent_t ev = nullptr;
    std::vector<std::pair<Tile*, int64_t>> parts;
};

size_t tile_bytes(const Dict& d, int64_t P, int K) {
    return align_up((size_t)P * d.M * 4, 256) + align_up((size_t)P * d.N * 4, 256) +
           align_up((size_t)P * K * 4, 256) + align_up((size_t)P * sizeof(csrec_pixel_stats), 256);
}

size_t result_bytes(const Dict& d, int64_t P, int K) {
    return align_up((size_t)P * d.N * 4, 256) + align_up((size_t)P * K * 4, 256) +
           align_up((size_t)P * sizeof(csrec_pixel_stats), 256);
}

// Pinned host staging: the device budget, at least 64 MiB and at most 4 GiB.
size_t host_pool_bytes(size_t hbm_budget) {
    const size_t lo = (size_t)64 << 20, hi = (size_t)4 << 30;
    return hbm_budget < lo ? lo : (hbm_budget > hi ? hi : hbm_budget);
}

}  // namespace
}  // namespace csrec

struct csrec_server {
    csrec_server_cfg cfg{};
    std::chrono::steady_clock::time_point t0;
    hipStream_t compute = nullptr, h2d = nullptr, d2h = nullptr;
    char* pool_mem = nullptr;
    char* host_mem = nullptr;             // pinned staging for inputs and results
    csrec::Pool hpool;
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
    std::vector<std::unique_ptr<csrec::Tile>> admitted;  // on the device, chunks being solved
    std::deque<std::unique_ptr<csrec::Tile>> computed;   // solved, waiting for host result memory
    std::vector<std::unique_ptr<csrec::Tile>> copying;   // result copy in flight
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

// Starts the result copy of a solved tile into pinned host memory; false
// when the host pool is momentarily full (retried on a later step).  A tile
// whose results could never fit the pool is copied into pageable vectors.
bool start_output(csrec_server* s, Tile* t) {
    const Dict& d = s->dicts[t->dict];
    const int K = s->cfg.gomp.K;
    const size_t bytes = result_bytes(d, t->P, K);
    char* h = s->hpool.alloc(bytes);
    if (!h && bytes <= s->hpool.capacity()) return false;
    if (h) {
        t->hout = h;
        t->X = reinterpret_cast<float*>(h);
        t->S = reinterpret_cast<int32_t*>(h + align_up((size_t)t->P * d.N * 4, 256));
        t->St = reinterpret_cast<csrec_pixel_stats*>(reinterpret_cast<char*>(t->S) + align_up((size_t)t->P * K * 4, 256));
    } else {
        t->Xv.resize((size_t)t->P * d.N);
        t->Sv.resize((size_t)t->P * K);
        t->Stv.resize((size_t)t->P);
        t->X = t->Xv.data();
        t->S = t->Sv.data();
        t->St = t->Stv.data();
    }
    hipError_t e = hipEventCreateWithFlags(&t->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemcpyAsync(t->X, t->dX, (size_t)t->P * d.N * 4, hipMemcpyDeviceToHost, s->d2h);
    if (e == hipSuccess) e = hipMemcpyAsync(t->S, t->dS, (size_t)t->P * K * 4, hipMemcpyDeviceToHost, s->d2h);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t->St, t->dSt, (size_t)t->P * sizeof(csrec_pixel_stats), hipMemcpyDeviceToHost, s->d2h);
    if (e == hipSuccess) e = hipEventRecord(t->ev_out, s->d2h);
    if (e != hipSuccess) {
        set_hip_error(e);
        s->error = CSREC_E_DEVICE;
        t->status = CSREC_E_DEVICE;
    }
    return true;
}

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
        for (auto& pr : b.parts) pr.first->done += pr.second;
        hipEventDestroy(b.ev);
        s->inflight.pop_front();
        worked = true;
    }
    // ---- solved tiles leave the admitted set in order of admission
    for (auto it = s->admitted.begin(); it != s->admitted.end();) {
        if ((*it)->done == (*it)->P) {
            s->computed.push_back(std::move(*it));
            it = s->admitted.erase(it);
            worked = true;
        } else {
            ++it;
        }
    }
    while (!s->computed.empty() && start_output(s, s->computed.front().get())) {
        s->copying.push_back(std::move(s->computed.front()));
        s->computed.pop_front();
        worked = true;
    }
    // ---- result copies that completed
    for (auto it = s->copying.begin(); it != s->copying.end();) {
        Tile* t = it->get();
        const hipError_t q = hipEventQuery(t->ev_out);
        if (q == hipErrorNotReady) {
            ++it;
            continue;
        }
        if (q != hipSuccess) {
            set_hip_error(q);
            s->error = CSREC_E_DEVICE;
            t->status = CSREC_E_DEVICE;
        }
        t->t_done = now_since(s->t0);
        s->pool.release(t->mem);
        t->mem = nullptr;
        if (t->hin) s->hpool.release(t->hin);
        t->hin = nullptr;
        std::vector<float>().swap(t->Yv);
        --s->outstanding;
        s->finished.push_back(std::move(*it));
        it = s->copying.erase(it);
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
        const void* src = t->hin ? static_cast<const void*>(t->hin) : static_cast<const void*>(t->Yv.data());
        hipError_t e = hipEventCreateWithFlags(&t->ev_in, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMemcpyAsync(t->dY, src, (size_t)t->P * d.M * 4, hipMemcpyHostToDevice, s->h2d);
        if (e == hipSuccess) e = hipEventRecord(t->ev_in, s->h2d);
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
            hipError_t he = hipSuccess;
            for (auto& pr : b.parts) {
                Tile* t = pr.first;
                if (!t->in_waited && he == hipSuccess) {
                    he = hipStreamWaitEvent(s->compute, t->ev_in, 0);
                    t->in_waited = true;
                }
            }
            int e = greedy_group_launch(s->proto, items.data(), (int)items.size(), s->cfg.batch_pixels, s->ws,
                                        s->table_host[s->table_flip], s->table_dev, s->compute);
            s->table_flip ^= 1;
            if (he == hipSuccess) he = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
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

// Releases a tile's host and device resources (lock held).
void drop_tile(csrec_server* s, Tile* t) {
    if (t->mem) s->pool.release(t->mem);
    if (t->hin) s->hpool.release(t->hin);
    if (t->hout) s->hpool.release(t->hout);
    if (t->ev_in) hipEventDestroy(t->ev_in);
    if (t->ev_out) hipEventDestroy(t->ev_out);
    t->mem = t->hin = t->hout = nullptr;
    t->ev_in = t->ev_out = nullptr;
}

void scheduler(csrec_server* s) {
    hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        if (s->stop && s->pending.empty() && s->admitted.empty() && s->computed.empty() && s->copying.empty() &&
            s->inflight.empty())
            break;
        if (s->error != CSREC_OK && s->inflight.empty()) {
            // fail every queued tile and stop issuing work
            for (auto& t : s->pending) {
                t->status = s->error;
                --s->outstanding;
                s->finished.push_back(std::move(t));
            }
            s->pending.clear();
            hipStreamSynchronize(s->h2d);
            hipStreamSynchronize(s->d2h);
            for (auto* lst : {&s->admitted, &s->copying}) {
                for (auto& t : *lst) {
                    t->status = s->error;
                    if (t->mem) s->pool.release(t->mem);
                    t->mem = nullptr;
                    --s->outstanding;
                    s->finished.push_back(std::move(t));
                }
                lst->clear();
            }
            for (auto& t : s->computed) {
                t->status = s->error;
                if (t->mem) s->pool.release(t->mem);
                t->mem = nullptr;
                --s->outstanding;
                s->finished.push_back(std::move(t));
            }
            s->computed.clear();
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
    if (g.S * p.max_iter > GOMP_CMAX || g.K > GOMP_CMAX) return CSREC_E_SHAPE;
    p.prune = g.prune;
    p.prec = g.prec;
    p.res_tol = (float)g.res_tol;
    p.eps = (float)g.eps;
    p.pivot_fallback = g.pivot_fallback;
    s->ws_bytes = greedy_group_workspace(p, cfg->batch_pixels);
    s->max_items = (int)std::min<int64_t>(4096, cfg->batch_pixels);
    CSREC_HIP_TRY(hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking));
    CSREC_HIP_TRY(hipStreamCreateWithFlags(&s->h2d, hipStreamNonBlocking));
    CSREC_HIP_TRY(hipStreamCreateWithFlags(&s->d2h, hipStreamNonBlocking));
    CSREC_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&s->pool_mem), cfg->hbm_budget_bytes));
    const size_t hb = host_pool_bytes(cfg->hbm_budget_bytes);
    CSREC_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&s->host_mem), hb, hipHostMallocDefault));
    s->hpool.init(s->host_mem, hb);
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
        if (P > 0) t->hin = s->hpool.alloc((size_t)P * M * 4);
    }
    // copied outside the lock
    if (t->hin)
        std::memcpy(t->hin, Y_host, (size_t)P * M * 4);
    else
        t->Yv.assign(Y_host, Y_host + (size_t)P * M);
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
        r.X = t->X;
        r.support = t->S;
        r.stats = t->St;
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
    auto it = s->polled.find(tag);
    if (it != s->polled.end()) {
        drop_tile(s, it->second.get());
        s->polled.erase(it);
    }
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
    hipStreamSynchronize(s->h2d);
    hipStreamSynchronize(s->d2h);
    for (auto& kv : s->polled) drop_tile(s, kv.second.get());
    for (auto& t : s->finished) drop_tile(s, t.get());
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
    hipHostFree(s->host_mem);
    hipStreamDestroy(s->compute);
    hipStreamDestroy(s->h2d);
    hipStreamDestroy(s->d2h);
    delete s;
    return CSREC_OK;
}

}  // extern "C"
