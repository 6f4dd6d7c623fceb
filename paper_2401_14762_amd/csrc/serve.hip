// Serving runtime: continuous batching of cube tiles through gOMP (Alg. 3).
//
// The scheduling core (admission by device budget, batching, retirement,
// host staging) is serving::Scheduler in serve_policy.hpp; this file is its
// HIP executor and the C ABI around it.
//
// Executor.  Three non-blocking streams at the default priority: input
// copies (host to device), the batched solves, and result copies (device to
// host).  A batch's solve waits on the device for the input copies of its
// tiles; one batch is one persistent grouped launch of the on-chip gOMP
// kernel per parameter class and kernel variant (every item of every tile in
// it is claimed unit by unit by resident workgroups), followed, when the
// class has an FP64 fallback threshold, by the grouped FP64 redo of the
// pixels the FP32 pass flagged.  Each operation ends with an event that the
// scheduler polls; events are recycled.  Dictionaries (A, its copies for
// the on-chip kernel and its Gram matrix in FP32 and FP64) stay on the device
// from csrec_server_add_dict until destroy; the per-pixel state of a batch
// lives in the batch workspace.  After creation nothing is allocated on the
// device except dictionaries.
#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "serve_policy.hpp"

namespace csrec {
namespace {

constexpr int kMaxDicts = 64;

struct Dict {
    int M = 0, N = 0;
    float* A = nullptr;
    float* AT = nullptr;
    float* G32 = nullptr;
    double* G64 = nullptr;
};

void free_dict(Dict& d) {
    if (d.A) hipFree(d.A);
    if (d.AT) hipFree(d.AT);
    if (d.G32) hipFree(d.G32);
    if (d.G64) hipFree(d.G64);
    d = Dict{};
}

class HipExecutor : public serving::Executor {
   public:
    hipStream_t compute = nullptr, h2d = nullptr, d2h = nullptr;
    char* dev_base = nullptr;        // device pool
    char* host_base = nullptr;       // pinned host staging pool
    char* ws = nullptr;              // batch workspace
    char* table_dev = nullptr;       // launch item tables, two halves
    char* table_host[2] = {nullptr, nullptr};
    size_t table_bytes = 0;
    int flip = 0;
    int64_t batch_pixels = 0;
    GreedyLaunch proto{};            // layout of the batch workspace (maximal shape)
    const std::array<Dict, kMaxDicts>* dicts = nullptr;

    ~HipExecutor() override {
        for (auto& kv : live_) hipEventDestroy(kv.second);
        for (hipEvent_t e : spare_) hipEventDestroy(e);
    }

    int input_start(serving::Tile& t, uint64_t* h) override {
        const void* src = t.hin_pool ? static_cast<const void*>(host_base + t.hin_off)
                                     : static_cast<const void*>(t.hin_vec.data());
        hipError_t e = hipMemcpyAsync(dev_base + t.dev_off, src, (size_t)t.P * t.M * 4, hipMemcpyHostToDevice, h2d);
        if (e != hipSuccess) return fail(e);
        return record(h2d, h);
    }

    int launch(const std::vector<serving::Chunk>& chunks, uint64_t* h) override {
        // the solve waits for the input copies still in flight
        std::vector<uint64_t> waited;
        for (const auto& c : chunks) {
            const serving::Tile* t = c.tile;
            if (t->in_done || !t->ev_in) continue;
            if (std::find(waited.begin(), waited.end(), t->ev_in) != waited.end()) continue;
            waited.push_back(t->ev_in);
            hipError_t e = hipStreamWaitEvent(compute, live_.at(t->ev_in), 0);
            if (e != hipSuccess) return fail(e);
        }
        char* thost = table_host[flip];
        char* tdev = table_dev + (size_t)flip * table_bytes;
        flip ^= 1;
        size_t off = 0;
        size_t i = 0;
        while (i < chunks.size()) {
            // one parameter class: chunks[i, j)
            size_t j = i + 1;
            while (j < chunks.size() && chunks[j].tile->prm.same_launch(chunks[i].tile->prm)) ++j;
            const serving::TileParams& prm = chunks[i].tile->prm;
            std::vector<GreedyTileItem> items;
            items.reserve(j - i);
            for (size_t k = i; k < j; ++k) {
                const serving::Tile* t = chunks[k].tile;
                const Dict& d = (*dicts)[t->dict];
                char* blk = dev_base + t->dev_off;
                GreedyTileItem it{};
                it.A = d.A;
                it.dict = d.AT;
                it.Y = reinterpret_cast<const float*>(blk);
                it.X = reinterpret_cast<float*>(blk + t->dev_x());
                it.support = reinterpret_cast<int32_t*>(blk + t->dev_s());
                it.stats = reinterpret_cast<csrec_pixel_stats*>(blk + t->dev_st());
                it.G32 = d.G32;
                it.G64 = d.G64;
                it.M = d.M;
                it.N = d.N;
                it.max_iter = t->prm.max_iter;
                it.p0 = chunks[k].p0;
                it.np = chunks[k].np;
                items.push_back(it);
            }
            GreedyLaunch pm = proto;
            pm.prune = prm.prune;
            pm.prec = prm.prec;
            pm.res_tol = prm.res_tol;
            pm.eps = prm.eps;
            pm.pivot_fallback = prm.pivot_fallback;
            pm.redo_tol = prm.redo_tol;
            const int e = greedy_group_launch(pm, items.data(), (int)items.size(), batch_pixels, ws, thost + off,
                                              tdev + off, compute);
            if (e) return e;
            off += align_up(greedy_group_table_bytes((int)items.size()), 256);
            i = j;
        }
        return record(compute, h);
    }

    int output_start(serving::Tile& t, uint64_t* h) override {
        char* dst = t.hout_pool ? host_base + t.hout_off : t.hout_vec.data();
        const char* blk = dev_base + t.dev_off;
        hipError_t e = hipMemcpyAsync(dst, blk + t.dev_x(), (size_t)t.P * t.N * 4, hipMemcpyDeviceToHost, d2h);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst + t.out_s(), blk + t.dev_s(), (size_t)t.P * t.prm.K * 4, hipMemcpyDeviceToHost,
                               d2h);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst + t.out_st(), blk + t.dev_st(), (size_t)t.P * sizeof(csrec_pixel_stats),
                               hipMemcpyDeviceToHost, d2h);
        if (e != hipSuccess) return fail(e);
        return record(d2h, h);
    }

    int query(uint64_t h) override {
        auto it = live_.find(h);
        if (it == live_.end()) return CSREC_E_INVAL;
        const hipError_t q = hipEventQuery(it->second);
        if (q == hipSuccess) return 0;
        if (q == hipErrorNotReady) return 1;
        return fail(q);
    }

    void forget(uint64_t h) override {
        auto it = live_.find(h);
        if (it == live_.end()) return;
        spare_.push_back(it->second);
        live_.erase(it);
    }

    char* host_ptr(size_t off) override { return host_base + off; }

    void wait_idle() override {
        hipStreamSynchronize(h2d);
        hipStreamSynchronize(compute);
        hipStreamSynchronize(d2h);
    }

   private:
    static int fail(hipError_t e) {
        set_hip_error(e);
        return CSREC_E_DEVICE;
    }
    int record(hipStream_t s, uint64_t* h) {
        hipEvent_t ev = nullptr;
        if (!spare_.empty()) {
            ev = spare_.back();
            spare_.pop_back();
        } else {
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return fail(e);
        }
        hipError_t e = hipEventRecord(ev, s);
        if (e != hipSuccess) {
            spare_.push_back(ev);
            return fail(e);
        }
        *h = next_++;
        live_[*h] = ev;
        return CSREC_OK;
    }
    std::map<uint64_t, hipEvent_t> live_;
    std::vector<hipEvent_t> spare_;
    uint64_t next_ = 1;
};

// Pinned host staging: the device budget, at least 64 MiB and at most 4 GiB.
size_t host_pool_bytes(size_t hbm_budget) {
    const size_t lo = (size_t)64 << 20, hi = (size_t)4 << 30;
    return hbm_budget < lo ? lo : (hbm_budget > hi ? hi : hbm_budget);
}

int check_gomp_params(const csrec_gomp_params& g) {
    if (g.struct_size != (int32_t)sizeof(csrec_gomp_params)) return CSREC_E_INVAL;
    if (g.K < 1 || g.S < 1 || g.S > 8 || g.max_iter < 0) return CSREC_E_INVAL;
    if (g.prune != CSREC_PRUNE_EACH && g.prune != CSREC_PRUNE_FINAL) return CSREC_E_INVAL;
    if (!(g.res_tol >= 0) || !(g.eps >= 0) || !(g.pivot_fallback >= 0) || !(g.redo_tol >= 0) ||
        !std::isfinite(g.redo_tol))
        return CSREC_E_INVAL;
    if (g.prec != CSREC_PREC_F32 && g.prec != CSREC_PREC_BF16 && g.prec != CSREC_PREC_F16) return CSREC_E_INVAL;
    return CSREC_OK;
}

}  // namespace
}  // namespace csrec

struct csrec_server {
    csrec_server_cfg cfg{};
    csrec::HipExecutor ex;
    std::unique_ptr<csrec::serving::Scheduler> sch;
    std::array<csrec::Dict, csrec::kMaxDicts> dicts{};
    std::atomic<int> ndicts{0};
    std::mutex dict_mu;
    int imax_cap = 0;                     // largest max_iter the batch workspace is laid out for
};

using namespace csrec;

namespace {

// Frees everything the server holds (any subset may be allocated).
void server_free(csrec_server* s) {
    if (!s) return;
    if (s->sch) s->sch->shutdown();
    s->sch.reset();
    hipSetDevice(s->cfg.device);
    for (auto& d : s->dicts) free_dict(d);
    HipExecutor& x = s->ex;
    if (x.dev_base) hipFree(x.dev_base);
    if (x.ws) hipFree(x.ws);
    if (x.table_dev) hipFree(x.table_dev);
    if (x.table_host[0]) hipHostFree(x.table_host[0]);
    if (x.table_host[1]) hipHostFree(x.table_host[1]);
    if (x.host_base) hipHostFree(x.host_base);
    if (x.compute) hipStreamDestroy(x.compute);
    if (x.h2d) hipStreamDestroy(x.h2d);
    if (x.d2h) hipStreamDestroy(x.d2h);
    delete s;
}

// The server's parameters with a tile's overrides, checked against the
// batch workspace: K and S must be the server's; max_iter may be smaller;
// an FP64 fallback needs a server created with one.
int resolve_params(const csrec_server* s, const csrec::Dict& d, const csrec_gomp_params* q,
                   serving::TileParams* out) {
    const csrec_gomp_params& g = q ? *q : s->cfg.gomp;
    int e = check_gomp_params(g);
    if (e) return e;
    if (g.K != s->cfg.gomp.K || g.S != s->cfg.gomp.S) return CSREC_E_UNSUPPORTED;
    if (g.pivot_fallback > 0 && !(s->cfg.gomp.pivot_fallback > 0)) return CSREC_E_UNSUPPORTED;
    const int imax = g.max_iter > 0 ? g.max_iter : std::min(g.K, d.M / g.S);
    if (imax < 1 || g.S * imax > d.M || imax > s->imax_cap) return CSREC_E_SHAPE;
    if (gomp_coop_supported(d.M, d.N, g.K, g.S, imax) != CSREC_OK) return CSREC_E_UNSUPPORTED;
    out->K = g.K;
    out->S = g.S;
    out->max_iter = imax;
    out->prune = g.prune;
    out->prec = g.prec;
    out->res_tol = (float)g.res_tol;
    out->eps = (float)g.eps;
    out->pivot_fallback = g.pivot_fallback;
    out->redo_tol = g.redo_tol > 0.0 ? g.redo_tol : CSREC_REDO_TOL_DEFAULT;
    return CSREC_OK;
}

}  // namespace

extern "C" {

int32_t csrec_server_create(const csrec_server_cfg* cfg, csrec_server** out) {
    if (!cfg || !out || cfg->struct_size != (int32_t)sizeof(csrec_server_cfg)) return CSREC_E_INVAL;
    const csrec_gomp_params& g = cfg->gomp;
    int e = check_gomp_params(g);
    if (e) return e;
    if (cfg->hbm_budget_bytes < 4096 || cfg->batch_pixels < 256 || cfg->chunk_pixels < 1) return CSREC_E_INVAL;
    const int imax = g.max_iter > 0 ? g.max_iter : std::min(g.K, 96 / g.S);
    if (g.S * imax > GOMP_CMAX || g.K > GOMP_CMAX) return CSREC_E_SHAPE;
    csrec_server* s = new csrec_server();
    s->cfg = *cfg;
    s->imax_cap = imax;
    HipExecutor& x = s->ex;
    x.dicts = &s->dicts;
    x.batch_pixels = cfg->batch_pixels;
    // the batch workspace is laid out for the largest shape a dictionary may have
    GreedyLaunch& p = x.proto;
    p.kind = GREEDY_GOMP;
    p.M = 96;
    p.N = CSREC_MAX_N;
    p.K = g.K;
    p.S = g.S;
    p.max_iter = imax;
    p.prune = g.prune;
    p.prec = g.prec;
    p.res_tol = (float)g.res_tol;
    p.eps = (float)g.eps;
    p.pivot_fallback = g.pivot_fallback;
    p.redo_tol = g.redo_tol > 0.0 ? g.redo_tol : CSREC_REDO_TOL_DEFAULT;
    const size_t ws_bytes = greedy_group_workspace(p, cfg->batch_pixels);
    const int max_items = (int)std::min<int64_t>(4096, cfg->batch_pixels);
    // every parameter class of a batch takes its own slice of the table
    x.table_bytes = align_up(greedy_group_table_bytes(max_items), 256) + (size_t)max_items * 2048;
    const size_t hb = host_pool_bytes(cfg->hbm_budget_bytes);
    hipError_t he = hipSetDevice(cfg->device);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&x.compute, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&x.h2d, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&x.d2h, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipMalloc(reinterpret_cast<void**>(&x.dev_base), cfg->hbm_budget_bytes);
    if (he == hipSuccess) he = hipHostMalloc(reinterpret_cast<void**>(&x.host_base), hb, hipHostMallocDefault);
    if (he == hipSuccess) he = hipMalloc(reinterpret_cast<void**>(&x.ws), ws_bytes);
    if (he == hipSuccess) he = hipMalloc(reinterpret_cast<void**>(&x.table_dev), 2 * x.table_bytes);
    if (he == hipSuccess)
        he = hipHostMalloc(reinterpret_cast<void**>(&x.table_host[0]), x.table_bytes, hipHostMallocDefault);
    if (he == hipSuccess)
        he = hipHostMalloc(reinterpret_cast<void**>(&x.table_host[1]), x.table_bytes, hipHostMallocDefault);
    if (he != hipSuccess) {
        set_hip_error(he);
        server_free(s);
        return CSREC_E_DEVICE;
    }
    serving::Config sc;
    sc.dev_bytes = cfg->hbm_budget_bytes;
    sc.host_bytes = hb;
    sc.batch_pixels = cfg->batch_pixels;
    sc.chunk_pixels = cfg->chunk_pixels;
    sc.max_items = max_items;
    sc.max_inflight = 2;
    s->sch.reset(new serving::Scheduler(sc, &s->ex));
    s->sch->start();
    *out = s;
    return CSREC_OK;
}

int32_t csrec_server_add_dict(csrec_server* s, const float* A_host, int32_t M, int32_t N, int32_t* dict_id) {
    if (!s || !A_host || !dict_id) return CSREC_E_INVAL;
    if (M < 1 || M >= N || N > CSREC_MAX_N) return CSREC_E_SHAPE;
    if (M > 96) return CSREC_E_UNSUPPORTED;
    const csrec_gomp_params& g = s->cfg.gomp;
    const int imax = g.max_iter > 0 ? g.max_iter : std::min(g.K, M / g.S);
    if (imax < 1 || g.S * imax > M || imax > s->imax_cap) return CSREC_E_SHAPE;
    if (gomp_coop_supported(M, N, g.K, g.S, imax) != CSREC_OK) return CSREC_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(s->dict_mu);
    const int id = s->ndicts.load(std::memory_order_relaxed);
    if (id >= kMaxDicts) return CSREC_E_INVAL;
    Dict d;
    d.M = M;
    d.N = N;
    hipStream_t st = nullptr;
    hipError_t e = hipSetDevice(s->cfg.device);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.A), (size_t)M * N * 4);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.G32), (size_t)N * N * 4);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.AT), gomp_coop_dict_floats(M, N) * 4);
    if (e == hipSuccess && g.pivot_fallback > 0) e = hipMalloc(reinterpret_cast<void**>(&d.G64), (size_t)N * N * 8);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemcpyAsync(d.A, A_host, (size_t)M * N * 4, hipMemcpyHostToDevice, st);
    int rc = CSREC_OK;
    if (e == hipSuccess) rc = greedy_gram(d.A, M, N, d.G32, d.G64, st);
    if (e == hipSuccess && rc == CSREC_OK) {
        gomp_coop_prepare(d.A, M, N, d.AT, st);
        e = hipGetLastError();
    }
    if (st) {
        const hipError_t e2 = hipStreamSynchronize(st);
        if (e == hipSuccess) e = e2;
        hipStreamDestroy(st);
    }
    if (e != hipSuccess || rc != CSREC_OK) {
        if (e != hipSuccess) set_hip_error(e);
        free_dict(d);
        return e != hipSuccess ? CSREC_E_DEVICE : rc;
    }
    s->dicts[id] = d;
    s->ndicts.store(id + 1, std::memory_order_release);
    *dict_id = id;
    return CSREC_OK;
}

int32_t csrec_server_submit(csrec_server* s, int32_t dict_id, const float* Y_host, int64_t P,
                            const csrec_gomp_params* params, uint64_t tag) {
    if (!s || (P > 0 && !Y_host) || P < 0) return CSREC_E_INVAL;
    if (dict_id < 0 || dict_id >= s->ndicts.load(std::memory_order_acquire)) return CSREC_E_INVAL;
    const Dict& d = s->dicts[dict_id];
    serving::TileParams prm;
    const int e = resolve_params(s, d, params, &prm);
    if (e) return e;
    return s->sch->submit(dict_id, d.M, d.N, prm, Y_host, P, tag);
}

int32_t csrec_server_poll(csrec_server* s, csrec_result* out, int32_t max, int32_t* n) {
    if (!s || !n || (max > 0 && !out)) return CSREC_E_INVAL;
    std::vector<const serving::Tile*> got;
    s->sch->poll(got, max);
    for (size_t k = 0; k < got.size(); ++k) {
        const serving::Tile* t = got[k];
        csrec_result& r = out[k];
        r.tag = t->tag;
        r.status = t->status;
        r.dict_id = t->dict;
        r.P = t->P;
        r.N = t->N;
        r.K = t->prm.K;
        char* base = t->status == CSREC_OK ? s->sch->results(t) : nullptr;
        r.X = base ? reinterpret_cast<const float*>(base) : nullptr;
        r.support = base ? reinterpret_cast<const int32_t*>(base + t->out_s()) : nullptr;
        r.stats = base ? reinterpret_cast<const csrec_pixel_stats*>(base + t->out_st()) : nullptr;
        r.t_submit = t->t_submit;
        r.t_admit = t->t_admit;
        r.t_done = t->t_done;
    }
    *n = (int32_t)got.size();
    return CSREC_OK;
}

int32_t csrec_server_release(csrec_server* s, uint64_t tag) {
    if (!s) return CSREC_E_INVAL;
    return s->sch->release(tag);
}

int32_t csrec_server_drain(csrec_server* s) {
    if (!s) return CSREC_E_INVAL;
    return s->sch->drain();
}

int32_t csrec_server_get_stats(csrec_server* s, csrec_server_stats* out) {
    if (!s || !out || out->struct_size != (int32_t)sizeof(csrec_server_stats)) return CSREC_E_INVAL;
    const serving::Counters c = s->sch->counters();
    out->tiles_submitted = c.tiles_submitted;
    out->tiles_finished = c.tiles_finished;
    out->batches = c.batches;
    out->pixels_launched = c.pixels_launched;
    out->host_in_pageable = c.host_in_pageable;
    out->host_out_pageable = c.host_out_pageable;
    out->elapsed_s = c.elapsed_s;
    out->busy_s = c.busy_s;
    out->mean_pixels_in_flight = c.elapsed_s > 0 ? c.slot_px_s / c.elapsed_s : 0.0;
    out->mean_pool_bytes = c.elapsed_s > 0 ? c.pool_bytes_s / c.elapsed_s : 0.0;
    return CSREC_OK;
}

int32_t csrec_server_destroy(csrec_server* s) {
    if (!s) return CSREC_E_INVAL;
    server_free(s);
    return CSREC_OK;
}

}  // extern "C"
