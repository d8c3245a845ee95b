// Request server: continuous (iteration-level) batching of generation
// requests with mixed grids on one GPU.
//
// Requests wait in a FIFO until a slot is free and their workspace fits in
// the server's device arena (admission by HBM footprint).  Each scheduling
// step takes pair-sum work items from the active requests -- those with the
// least work left first (or round-robin), enough to fill the GPU a couple of
// times over -- and runs them in one persistent launch; a request admitted
// between steps joins the next one.  A
// request whose plan uses the pair sum through a DFT along kappa runs that
// whole stage at admission, on the step's lane; a request with zero
// bicoherence has no pair stage.  A
// request whose items have all been issued gets its transforms and a
// completion event; its slot and arena space are released when that event
// has completed.  Per-step tables travel in one host-to-device copy from a
// pinned staging buffer.  Consecutive steps alternate between two streams,
// each with its own staging buffers, so that a step's items start on compute
// units the previous step's longest items leave idle; events order a
// request's phases before its items and all its items before its transforms.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "srm3_internal.hpp"

using namespace srm3;

namespace {

// Per-slot header read by the kernels of a request (device copy of the table).
struct SlotHeader {
    uint64_t seed;
    double scale;
    const double *S;   // device spectrum or null (plan's)
    void *out;
};

struct Item {
    int kb, cg;
    double cost;
};

struct SReq {
    int64_t ticket = 0;
    srm3_request r{};
    bool own_spec = false;
    srm3_kaimal_davenport spec{};
    Geometry g{};
    size_t off = 0, bytes = 0;      // arena slice: workspace [+ spectrum]
    int slot = -1;
    bool fresh = false;             // admitted, phases not yet launched
    int mode = 0;                   // 0: pair-sum items in the persistent launch; 1: the plan's kappa-DFT
                                    // pair sum, run at admission; 2: zero bicoherence, no pair sum
    size_t kfft_off = 0;            // arena offset of the kappa-DFT workspace (mode 1)
    std::vector<Item> items;        // heaviest first
    size_t cursor = 0;
    double left = 0.0;              // cost of the items not yet issued
    hipEvent_t done = nullptr;
};

// First-fit allocator over [0, size) with coalescing.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void reset(size_t n)
    {
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = (n + 255) & ~static_cast<size_t>(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, noff = it->first + n;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + 255) & ~static_cast<size_t>(255);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

}  // namespace

struct srm3_server_s {
    srm3_server_config cfg{};
    hipStream_t st = nullptr;           // caller's stream (ordering at creation and destruction)
    hipStream_t lane[2] = {nullptr, nullptr};
    hipEvent_t ev_phases[2] = {nullptr, nullptr}, ev_pairsum[2] = {nullptr, nullptr};
    bool recorded[2] = {false, false};
    int R = 16;
    int n_cu = 256;
    int blocks_per_cu = 2;
    bool mfma = false;                 // persistent launch with matrix-core items
    int mfma_shape = 0;                // their tile shape
    DevBuf arena_mem;
    Arena arena;
    // staging: headers | qbegin | preq | items
    size_t off_hdr = 0, off_q = 0, off_req = 0, off_items = 0, stage_bytes = 0;
    int max_items = 0;
    DevBuf dev_stage[2], qnext[2];
    unsigned char *pinned[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    bool copy_pending[2] = {false, false};
    hipEvent_t step_done[2] = {nullptr, nullptr};
    bool step_pending[2] = {false, false};
    int cur = 0;
    std::vector<SlotHeader> hdr;               // host mirror
    std::vector<unsigned char> preq;           // host mirror, one PReq per slot
    std::vector<SReq *> slot_req;              // active requests by slot
    std::vector<SReq *> order;                 // active in admission order
    std::deque<SReq *> queue;
    std::vector<SReq *> finishing;
    std::deque<int64_t> completed;
    std::vector<hipEvent_t> ev_pool;
    int64_t next_ticket = 1;
    int64_t steps = 0;
};

namespace {

srm3_status take_event(srm3_server_t s, hipEvent_t *ev)
{
    if (!s->ev_pool.empty()) {
        *ev = s->ev_pool.back();
        s->ev_pool.pop_back();
        return SRM3_OK;
    }
    hipError_t e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    return e == hipSuccess ? SRM3_OK : dev_err(e, "hipEventCreate");
}

size_t request_bytes(const srm3_server_s *s, const Geometry &g, bool own_spec)
{
    size_t b = align256(workspace_bytes(g, s->cfg.precision, 1));
    if (own_spec) b += align256(static_cast<size_t>(g.nk) * g.nc * sizeof(double));
    return b;
}

void free_request(srm3_server_t s, SReq *q)
{
    if (q->slot >= 0) {
        s->slot_req[q->slot] = nullptr;
        s->hdr[q->slot] = SlotHeader{};
    }
    if (q->bytes) s->arena.release(q->off, q->bytes);
    if (q->done) s->ev_pool.push_back(q->done);
    delete q;
}

// Retire requests whose completion event has fired.
srm3_status retire(srm3_server_t s)
{
    for (size_t i = 0; i < s->finishing.size();) {
        SReq *q = s->finishing[i];
        const hipError_t e = hipEventQuery(q->done);
        if (e == hipErrorNotReady) {
            ++i;
            continue;
        }
        if (e != hipSuccess) return dev_err(e, "hipEventQuery");
        s->completed.push_back(q->ticket);
        s->finishing.erase(s->finishing.begin() + static_cast<long>(i));
        free_request(s, q);
    }
    return SRM3_OK;
}

}  // namespace

extern "C" {

srm3_status srm3_server_create(const srm3_server_config *cfg, void *hip_stream, srm3_server_t *out)
{
    if (!out) return fail(SRM3_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(SRM3_E_INVALID, "config is NULL");
    if (cfg->precision != SRM3_FP32 && cfg->precision != SRM3_FP64)
        return fail(SRM3_E_INVALID, "precision %d", cfg->precision);
    if (cfg->max_active < 1 || cfg->max_active > 4096) return fail(SRM3_E_INVALID, "max_active %d", cfg->max_active);
    if (cfg->hbm_budget < (1u << 16)) return fail(SRM3_E_INVALID, "hbm_budget below 64 KiB");
    if (cfg->policy != SRM3_SERVE_SHORTEST_FIRST && cfg->policy != SRM3_SERVE_ROUND_ROBIN)
        return fail(SRM3_E_INVALID, "policy %d", cfg->policy);
    if (cfg->pair_kernel != SRM3_ALGO_DIRECT && cfg->pair_kernel != SRM3_ALGO_MFMA)
        return fail(SRM3_E_INVALID, "pair_kernel %d", cfg->pair_kernel);
    if (cfg->mfma_shape < 0 || cfg->mfma_shape >= kMfmaShapes)
        return fail(SRM3_E_INVALID, "mfma_shape %d", cfg->mfma_shape);
    std::unique_ptr<srm3_server_s> s(new (std::nothrow) srm3_server_s);
    if (!s) return fail(SRM3_E_NOMEM, "host allocation failed");
    s->cfg = *cfg;
    if (!(s->cfg.step_pair_terms > 0)) s->cfg.step_pair_terms = 2e11;
    s->st = static_cast<hipStream_t>(hip_stream);
    s->R = cfg->precision == SRM3_FP64 ? 8 : 16;
    s->mfma = cfg->pair_kernel == SRM3_ALGO_MFMA;
    s->mfma_shape = cfg->mfma_shape;
    if (s->mfma) s->blocks_per_cu = 3;   // the matrix-core kernel runs 3 waves per SIMD
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        s->n_cu = prop.multiProcessorCount;
    hipError_t e = s->arena_mem.alloc(cfg->hbm_budget);
    if (e != hipSuccess) return fail(SRM3_E_NOMEM, "arena hipMalloc(%zu): %s", cfg->hbm_budget, hipGetErrorString(e));
    s->arena.reset(cfg->hbm_budget);
    const int na = cfg->max_active;
    s->max_items = 1 << 17;
    s->off_hdr = 0;
    s->off_q = align256(sizeof(SlotHeader) * na);
    s->off_req = s->off_q + align256(sizeof(int) * (kXcds + 1));
    s->off_items = s->off_req + align256(persistent_req_bytes() * na);
    s->stage_bytes = s->off_items + align256(persistent_item_bytes() * s->max_items);
    for (int i = 0; i < 2; ++i) {
        if ((e = s->dev_stage[i].alloc(s->stage_bytes)) != hipSuccess ||
            (e = s->qnext[i].alloc(kXcds * sizeof(int))) != hipSuccess)
            return fail(SRM3_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
        if ((e = hipStreamCreateWithFlags(&s->lane[i], hipStreamNonBlocking)) != hipSuccess)
            return dev_err(e, "hipStreamCreate");
        if ((e = hipEventCreateWithFlags(&s->ev_phases[i], hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s->ev_pairsum[i], hipEventDisableTiming)) != hipSuccess)
            return dev_err(e, "hipEventCreate");
    }
    // the arena and staging must be ready before work is enqueued on the lanes
    if ((e = hipDeviceSynchronize()) != hipSuccess) return dev_err(e, "hipDeviceSynchronize");
    for (int i = 0; i < 2; ++i) {
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&s->pinned[i]), s->stage_bytes, hipHostMallocDefault)) !=
            hipSuccess)
            return fail(SRM3_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
        if ((e = hipEventCreateWithFlags(&s->copied[i], hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s->step_done[i], hipEventDisableTiming)) != hipSuccess)
            return dev_err(e, "hipEventCreate");
    }
    s->hdr.assign(na, SlotHeader{});
    s->preq.assign(persistent_req_bytes() * na, 0);
    s->slot_req.assign(na, nullptr);
    *out = s.release();
    return SRM3_OK;
}

srm3_status srm3_server_submit(srm3_server_t s, const srm3_request *req, const srm3_kaimal_davenport *spectrum,
                               int64_t *ticket)
{
    if (!s || !req || !ticket) return fail(SRM3_E_INVALID, "NULL argument");
    const srm3_request &r = *req;
    if (!r.plan || !r.out_dev) return fail(SRM3_E_INVALID, "NULL plan or output");
    if (r.plan->precision != s->cfg.precision) return fail(SRM3_E_INVALID, "request precision differs from the server's");
    if (!(r.b2_scale > 0) || !std::isfinite(r.b2_scale)) return fail(SRM3_E_INVALID, "b2_scale must be finite and > 0");
    if (max_sigma(r.plan->max_sig, r.plan->cap, r.b2_scale) >= 1.0)
        return fail(SRM3_E_PURE_NEGATIVE, "scaled sum of b^2 reaches 1");
    if (spectrum && r.S_dev) return fail(SRM3_E_INVALID, "give either S_dev or spectrum parameters, not both");
    if (spectrum && (!(spectrum->U > 0) || !(spectrum->z > 0) || !(spectrum->lam > 0) || !(spectrum->u_star >= 0)))
        return fail(SRM3_E_INVALID, "bad spectrum parameters");
    if (r.plan->hashed) return fail(SRM3_E_UNSUPPORTED, "bispectra generated per pair run through srm3_generate");
    const bool kfft = r.plan->algo == SRM3_ALGO_KAPPA_FFT || r.plan->algo == SRM3_ALGO_FFT2D;
    if (!r.plan->gaussian && !kfft && (r.plan->algo == SRM3_ALGO_MFMA) != s->mfma)
        return fail(SRM3_E_UNSUPPORTED, "the server's direct-form pair sum runs on the %s: the plan's algorithm differs",
                    s->mfma ? "matrix cores" : "vector ALUs");
    if (r.plan->fixed_spectrum && (r.S_dev || spectrum))
        return fail(SRM3_E_UNSUPPORTED, "a product bispectrum's plan keeps its own spectrum");
    if (spectrum && r.plan->process)
        return fail(SRM3_E_UNSUPPORTED, "the wind spectrum is a wave spectrum; a process request takes S_dev");
    std::unique_ptr<SReq> q(new (std::nothrow) SReq);
    if (!q) return fail(SRM3_E_NOMEM, "host allocation failed");
    q->r = r;
    q->own_spec = spectrum != nullptr;
    if (spectrum) q->spec = *spectrum;
    q->g = r.plan->g;
    q->mode = r.plan->gaussian ? 2 : (kfft ? 1 : 0);
    if (q->mode == 0) {
        q->g.R = rows_for(q->g.nk, s->cfg.precision, s->R);
        // the vector kernel's persistent launch has one row count per wave; the
        // matrix-core items do not depend on it (it only pads the a planes)
        if (q->g.R != s->R && !s->mfma)
            return fail(SRM3_E_UNSUPPORTED, "grids with n_kappa < %d are not served", s->R);
        q->g.nkp = ((q->g.nk + q->g.R - 1) / q->g.R) * q->g.R;
    }
    q->bytes = request_bytes(s, q->g, q->own_spec);
    if (q->mode == 1) {
        q->kfft_off = q->bytes;
        q->bytes += align256(kfft_workspace_bytes(q->g, r.plan->kg, s->cfg.precision, 1));
    }
    if (q->bytes > s->arena.size)
        return fail(SRM3_E_NOMEM, "request needs %zu bytes, more than the server's budget %zu", q->bytes, s->arena.size);
    if (q->mode == 0) {
        const int mr = mfma_rows_per_group(s->cfg.precision, s->mfma_shape);
        const int mc = mfma_cols_per_group(s->cfg.precision, s->mfma_shape);
        const int nrb = s->mfma ? (q->g.nk + mr - 1) / mr : q->g.nkp / q->g.R;
        const int ncg = s->mfma ? (q->g.nc + mc - 1) / mc
                                : ((q->g.nc + 63) / 64 + waves_per_block() - 1) / waves_per_block();
        for (int kb = nrb - 1; kb >= 0; --kb)
            for (int cg = 0; cg < ncg; ++cg)
                q->items.push_back({kb, cg, s->mfma ? mfma_item_cost(q->g, kb, cg, s->cfg.precision, s->mfma_shape) : item_cost(q->g, q->g.R, kb, cg)});
        std::stable_sort(q->items.begin(), q->items.end(),
                         [](const Item &a, const Item &b) { return a.cost > b.cost; });
        for (const Item &it : q->items) q->left += it.cost;
        if (static_cast<int>(q->items.size()) > s->max_items) return fail(SRM3_E_UNSUPPORTED, "grid too large");
    }
    q->ticket = s->next_ticket++;
    *ticket = q->ticket;
    s->queue.push_back(q.release());
    return SRM3_OK;
}

srm3_status srm3_server_step(srm3_server_t s, srm3_server_state *state)
{
    if (!s) return fail(SRM3_E_INVALID, "server is NULL");
    srm3_status rc = retire(s);
    if (rc) return rc;
    // keep at most two steps in flight
    const int c = s->cur;
    bool launched = false;
    if (s->step_pending[c]) {
        const hipError_t e = hipEventQuery(s->step_done[c]);
        if (e == hipErrorNotReady) goto report;
        if (e != hipSuccess) return dev_err(e, "hipEventQuery");
        s->step_pending[c] = false;
    }
    {
        // ---- admission: FIFO, by free slot and arena space ----
        std::vector<SReq *> fresh;
        while (!s->queue.empty()) {
            SReq *q = s->queue.front();
            int slot = -1;
            for (int i = 0; i < s->cfg.max_active; ++i)
                if (!s->slot_req[i]) {
                    slot = i;
                    break;
                }
            if (slot < 0 || !s->arena.alloc(q->bytes, &q->off)) break;
            s->queue.pop_front();
            q->slot = slot;
            q->fresh = true;
            s->slot_req[slot] = q;
            s->order.push_back(q);
            char *base = static_cast<char *>(s->arena_mem.p) + q->off;
            const Workspace ws = carve_workspace(q->g, s->cfg.precision, 1, base);
            const double *S = q->r.S_dev;
            if (q->own_spec)
                S = reinterpret_cast<const double *>(base + align256(workspace_bytes(q->g, s->cfg.precision, 1)));
            s->hdr[slot] = SlotHeader{q->r.seed, q->r.b2_scale, S, q->r.out_dev};
            fill_persistent_req(s->preq.data() + persistent_req_bytes() * slot, q->g, ws.zrow, ws.zcol, ws.tsum,
                                q->r.plan->wtab.p);
            fresh.push_back(q);
        }
        // ---- this step's work: enough items to fill the GPU twice and meet the
        // pair-term budget, taken shortest-remaining-work first (or round-robin) ----
        std::vector<std::vector<Item>> take(s->order.size());
        const double unit = 64.0 * waves_per_block() * s->R;   // pair terms per unit of item cost
        const double budget = s->cfg.step_pair_terms / unit;
        const int min_items = 2 * s->n_cu * s->blocks_per_cu;
        double spent = 0.0;
        int n_items = 0;
        auto full = [&]() { return (spent >= budget && n_items >= min_items) || n_items >= s->max_items; };
        if (s->cfg.policy == SRM3_SERVE_SHORTEST_FIRST) {
            std::vector<size_t> pri(s->order.size());
            for (size_t i = 0; i < pri.size(); ++i) pri[i] = i;
            std::stable_sort(pri.begin(), pri.end(),
                             [&](size_t a, size_t b) { return s->order[a]->left < s->order[b]->left; });
            for (size_t i : pri) {
                SReq *q = s->order[i];
                while (q->cursor < q->items.size() && !full()) {
                    take[i].push_back(q->items[q->cursor++]);
                    spent += take[i].back().cost;
                    q->left -= take[i].back().cost;
                    ++n_items;
                }
                if (full()) break;
            }
        } else {
            bool more = true;
            while (more && !full()) {
                more = false;
                for (size_t i = 0; i < s->order.size() && !full(); ++i) {
                    SReq *q = s->order[i];
                    if (q->cursor >= q->items.size()) continue;
                    take[i].push_back(q->items[q->cursor++]);
                    spent += take[i].back().cost;
                    q->left -= take[i].back().cost;
                    ++n_items;
                    more = true;
                }
            }
        }
        if (fresh.empty() && n_items == 0) goto report;
        // ---- stage: headers, queues (requests kept contiguous, cut into per-XCD runs), items ----
        if (s->copy_pending[c]) {
            hipError_t e = hipEventSynchronize(s->copied[c]);
            if (e != hipSuccess) return dev_err(e, "hipEventSynchronize");
            s->copy_pending[c] = false;
        }
        unsigned char *P = s->pinned[c];
        std::memcpy(P + s->off_hdr, s->hdr.data(), sizeof(SlotHeader) * s->cfg.max_active);
        std::memcpy(P + s->off_req, s->preq.data(), s->preq.size());
        int *qb = reinterpret_cast<int *>(P + s->off_q);
        const size_t ib = persistent_item_bytes();
        int k = 0, q_ix = 1;
        double acc = 0.0;
        qb[0] = 0;
        for (size_t i = 0; i < take.size(); ++i)
            for (const Item &it : take[i]) {
                while (q_ix < kXcds && acc >= spent * q_ix / kXcds) qb[q_ix++] = k;
                fill_persistent_item(P + s->off_items + ib * k, s->order[i]->slot, it.kb, it.cg);
                acc += it.cost;
                ++k;
            }
        while (q_ix <= kXcds) qb[q_ix++] = k;
        const size_t bytes = s->off_items + ib * static_cast<size_t>(std::max(k, 1));
        hipStream_t st = s->lane[c];
        const int o = c ^ 1;
        hipError_t e = hipMemcpyAsync(s->dev_stage[c].p, P, bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return dev_err(e, "hipMemcpyAsync");
        if ((e = hipEventRecord(s->copied[c], st)) != hipSuccess) return dev_err(e, "hipEventRecord");
        s->copy_pending[c] = true;
        const SlotHeader *hdr_dev =
            reinterpret_cast<const SlotHeader *>(static_cast<char *>(s->dev_stage[c].p) + s->off_hdr);
        // ---- spectra and phases of the newly admitted requests ----
        for (SReq *q : fresh) {
            char *base = static_cast<char *>(s->arena_mem.p) + q->off;
            const Workspace ws = carve_workspace(q->g, s->cfg.precision, 1, base);
            if (q->own_spec) {
                const srm3_plan_t p = q->r.plan;
                e = launch_spectrum(q->g.nk, q->g.nw, p->dk, p->dw, q->spec.u_star, q->spec.z, q->spec.U,
                                    q->spec.lam, const_cast<double *>(s->hdr[q->slot].S), st);
                if (e != hipSuccess) return dev_err(e, "spectrum kernel");
            }
            Workspace wp = ws;
            if (q->mode != 0) wp.zcol = nullptr;   // no a operand planes needed
            e = launch_phases(q->g, s->cfg.precision, nullptr, &hdr_dev[q->slot].seed, 1, wp,
                              static_cast<const double *>(q->r.plan->lr.p), st);
            if (e != hipSuccess) return dev_err(e, "phase kernel");
            if (q->mode == 1) {
                // the whole pair sum of this request, here on the lane
                const srm3_plan_t p = q->r.plan;
                const KfftWorkspace kw = carve_kfft(q->g, p->kg, s->cfg.precision, 1, base + q->kfft_off);
                e = launch_kfft_pairsum(s->cfg.precision, q->g, p->kg, plan_ktab(p), 1, ws, kw, st);
                if (e != hipSuccess) return dev_err(e, "kappa-DFT pair-sum kernels");
            }
            q->fresh = false;
        }
        if ((e = hipEventRecord(s->ev_phases[c], st)) != hipSuccess) return dev_err(e, "hipEventRecord");
        // items may belong to requests admitted by the previous step on the other lane
        if (s->recorded[o] && (e = hipStreamWaitEvent(st, s->ev_phases[o], 0)) != hipSuccess)
            return dev_err(e, "hipStreamWaitEvent");
        // ---- pair sums ----
        if (k > 0) {
            char *D = static_cast<char *>(s->dev_stage[c].p);
            e = launch_pairsum_persistent(s->cfg.precision, s->R, D + s->off_req, D + s->off_items,
                                          reinterpret_cast<const int *>(D + s->off_q),
                                          static_cast<int *>(s->qnext[c].p), s->n_cu * s->blocks_per_cu, st, s->mfma,
                                          s->mfma_shape);
            if (e != hipSuccess) return dev_err(e, "persistent pair-sum kernel");
        }
        if ((e = hipEventRecord(s->ev_pairsum[c], st)) != hipSuccess) return dev_err(e, "hipEventRecord");
        bool waited = false;
        // ---- transforms of requests whose work has all been issued ----
        for (size_t i = 0; i < s->order.size();) {
            SReq *q = s->order[i];
            if (q->cursor < q->items.size()) {
                ++i;
                continue;
            }
            if (!waited && s->recorded[o]) {
                // earlier items of these requests may still run in the other lane's step
                if ((e = hipStreamWaitEvent(st, s->ev_pairsum[o], 0)) != hipSuccess)
                    return dev_err(e, "hipStreamWaitEvent");
                waited = true;
            }
            char *base = static_cast<char *>(s->arena_mem.p) + q->off;
            const Workspace ws = carve_workspace(q->g, s->cfg.precision, 1, base);
            AmpRef amp = plan_amp(q->r.plan);
            amp.scale_b = &hdr_dev[q->slot].scale;
            amp.S_b = &hdr_dev[q->slot].S;
            amp.tab = nullptr;   // per-realization scales and spectra: amplitudes per line
            e = launch_tfft(q->g, s->cfg.precision, 0, nullptr, amp, q->r.plan->wtab.p, q->r.plan->tw_t.p, 1, ws,
                            st);
            if (e != hipSuccess) return dev_err(e, "t-transform kernel");
            e = launch_xfft(q->g, s->cfg.precision, q->r.plan->tw_x.p, 1, ws, nullptr,
                            reinterpret_cast<void *const *>(&hdr_dev[q->slot].out), st);
            if (e != hipSuccess) return dev_err(e, "x-transform kernel");
            if ((rc = take_event(s, &q->done))) return rc;
            if ((e = hipEventRecord(q->done, st)) != hipSuccess) return dev_err(e, "hipEventRecord");
            s->finishing.push_back(q);
            s->order.erase(s->order.begin() + static_cast<long>(i));
        }
        if ((e = hipEventRecord(s->step_done[c], st)) != hipSuccess) return dev_err(e, "hipEventRecord");
        s->step_pending[c] = true;
        s->recorded[c] = true;
        s->cur ^= 1;
        ++s->steps;
        launched = true;
    }
report:
    if (state) {
        state->queued = static_cast<int32_t>(s->queue.size());
        state->active = static_cast<int32_t>(s->order.size());
        state->finishing = static_cast<int32_t>(s->finishing.size());
        state->completed = static_cast<int32_t>(s->completed.size());
        state->launched = launched ? 1 : 0;
        state->steps = s->steps;
    }
    return SRM3_OK;
}

srm3_status srm3_server_poll(srm3_server_t s, int64_t *tickets, int32_t max, int32_t *n)
{
    if (!s || !n || (max > 0 && !tickets)) return fail(SRM3_E_INVALID, "bad argument");
    srm3_status rc = retire(s);
    if (rc) return rc;
    int32_t k = 0;
    while (k < max && !s->completed.empty()) {
        tickets[k++] = s->completed.front();
        s->completed.pop_front();
    }
    *n = k;
    return SRM3_OK;
}

void srm3_server_destroy(srm3_server_t s)
{
    if (!s) return;
    for (int i = 0; i < 2; ++i)
        if (s->lane[i]) (void)hipStreamSynchronize(s->lane[i]);
    (void)hipDeviceSynchronize();
    for (SReq *q : s->queue) delete q;
    for (SReq *q : s->order) {
        if (q->done) (void)hipEventDestroy(q->done);
        delete q;
    }
    for (SReq *q : s->finishing) {
        if (q->done) (void)hipEventDestroy(q->done);
        delete q;
    }
    for (hipEvent_t ev : s->ev_pool) (void)hipEventDestroy(ev);
    for (int i = 0; i < 2; ++i) {
        if (s->pinned[i]) (void)hipHostFree(s->pinned[i]);
        for (hipEvent_t ev : {s->copied[i], s->step_done[i], s->ev_phases[i], s->ev_pairsum[i]})
            if (ev) (void)hipEventDestroy(ev);
        if (s->lane[i]) (void)hipStreamDestroy(s->lane[i]);
    }
    delete s;
}

}  // extern "C"
