// Serving scheduler of libdsdp: continuous batching of docking requests.
//
// Requests (receptor, ligand, chains, steps, seed) arrive at any time.  Each call
// of dsdp_sched_tick admits queued requests whose resources are free -- chain
// slots, arena space for the ligand blob and, when the receptor's maps are not
// resident, pool memory for them (evicting maps of receptors without running
// requests, least recently used first) -- then advances every running chain by
// one tick of MC steps in shared launches (one per pair-list size class), and
// ranks the requests whose chains finished.  All device memory comes from one
// caller-owned pool.  A request's chains run the same arithmetic as dsdp_dock
// on the same maps, so results do not depend on what else is in flight.
#include "../../include/dsdp.h"
#include "dsdp_host.h"
#include "dsdp_internal.h"
#include "range_alloc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

using namespace dsdp;
using namespace dsdp::host;

namespace {

constexpr int kMaxReceptors = 256;

struct Receptor {
    std::vector<dsdp_atom> atoms;
    dsdp_box box;
    std::vector<int32_t> types;
    int map_of_type[kNXS];
    std::vector<float4> site;   // search-space points (none: the whole box)
    float site_r = 0.f;
    bool resident = false;
    size_t maps_off = 0, maps_bytes = 0;   // maps, then the site points, in one pool range
    int active = 0;
    uint64_t last_use = 0;
};

enum { kQueued = 0, kRunning = 1, kDone = 2, kCancelled = 3 };

struct Request {
    int64_t ticket = 0;
    int receptor = 0;
    Prepared pl;
    int n_chains = 0, n_steps = 0, top_k = 0;
    uint64_t seed = 0;
    int state = kQueued;
    bool cancel = false;
    size_t slot0 = 0, arena_off = 0, arena_bytes = 0;
    int steps_done = 0;
    bool fresh = false;
    int passed_over = 0;     // admission rounds in which it did not fit
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<dsdp_pose> result;
    dsdp_dock_stats stats{};
};

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct dsdp_sched_s {
    char *pool = nullptr;
    size_t pool_bytes = 0;
    hipStream_t stream = nullptr;
    int capacity = 0, spt = 0;
    dsdp_params prm{};
    SearchParams sp{};
    RangeAlloc mem, slots;
    size_t off_tasks = 0, off_state = 0, off_records = 0, off_xyz = 0, off_segs = 0, off_sel = 0, off_grids = 0;
    std::vector<Receptor> receptors;
    std::vector<GridView> h_grids;
    bool grids_dirty = true;
    std::deque<Request *> queue;
    std::vector<Request *> running;
    std::deque<int64_t> finished;     // done or cancelled, not yet drained
    std::map<int64_t, std::unique_ptr<Request>> requests;
    int64_t next_ticket = 1;
    uint64_t clock = 0;
    double t0 = 0;
    int64_t map_builds = 0, evictions = 0, ticks = 0, completed = 0;
    std::vector<ChainTask> h_tasks;
    std::vector<RankSeg> h_segs;
};

namespace {

size_t fixed_bytes(int capacity)
{
    size_t b = 0;
    b += align256((size_t)capacity * sizeof(ChainTask));         // tasks
    b += align256((size_t)capacity * kStWords * 4);              // state
    b += align256((size_t)capacity * kRecWords * 4);             // records
    b += align256((size_t)capacity * kXyzStride * 16);           // best coordinates
    b += align256((size_t)capacity * sizeof(RankSeg));           // ranking segments
    b += align256((size_t)capacity * 2 * 4);                     // ranking output
    b += align256((size_t)kMaxReceptors * sizeof(GridView));     // grid views
    return b;
}

void evict(dsdp_sched s, Receptor &r)
{
    s->mem.release(r.maps_off, r.maps_bytes);
    r.resident = false;
    s->evictions++;
}

// Make receptor `id` resident, evicting idle receptors (LRU) when needed.
// Returns DSDP_OK, DSDP_ERR_BUSY when memory cannot be found now, or an error.
dsdp_status ensure_resident(dsdp_sched s, int id)
{
    Receptor &r = s->receptors[(size_t)id];
    if (r.resident) return DSDP_OK;
    const size_t maps_only = align256(dsdp_grids_bytes(&r.box, (int32_t)r.types.size()));
    const size_t maps = maps_only + align256(r.site.size() * sizeof(float4));
    const size_t wsb = align256(dsdp_build_grids_workspace_bytes((int32_t)r.atoms.size(), &r.box));
    size_t mo = 0, wo = 0;
    for (;;) {
        bool ok_m = s->mem.alloc(maps, mo);
        bool ok_w = ok_m && s->mem.alloc(wsb, wo);
        if (ok_m && ok_w) break;
        if (ok_m) s->mem.release(mo, maps);
        // evict the least recently used resident receptor with no running request
        int victim = -1;
        for (size_t k = 0; k < s->receptors.size(); k++) {
            const Receptor &c = s->receptors[k];
            if (c.resident && c.active == 0 && (victim < 0 || c.last_use < s->receptors[(size_t)victim].last_use))
                victim = (int)k;
        }
        if (victim < 0) return DSDP_ERR_BUSY;
        evict(s, s->receptors[(size_t)victim]);
    }
    dsdp_grids g = nullptr;
    dsdp_status st = dsdp_build_grids(r.atoms.data(), (int32_t)r.atoms.size(), &r.box, r.types.data(),
                                      (int32_t)r.types.size(), s->pool + mo, maps_only, s->pool + wo, wsb, s->stream,
                                      &g);
    if (st) {
        s->mem.release(mo, maps);
        s->mem.release(wo, wsb);
        return st;
    }
    hipError_t e = hipSuccess;
    if (!r.site.empty())
        e = hipMemcpyAsync(s->pool + mo + maps_only, r.site.data(), r.site.size() * sizeof(float4),
                           hipMemcpyHostToDevice, s->stream);
    // the build reads the workspace (and the copy the host points): wait before
    // handing them back
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    s->mem.release(wo, wsb);
    if (e != hipSuccess) {
        dsdp_grids_release(g);
        s->mem.release(mo, maps);
        return hip_fail(e, "map build");
    }
    GridView v = g->view;
    v.n_site = (int)r.site.size();
    v.site_r = r.site_r;
    v.site = v.n_site ? (const float4 *)(s->pool + mo + maps_only) : nullptr;
    s->h_grids[(size_t)id] = v;
    dsdp_grids_release(g);
    s->grids_dirty = true;
    r.resident = true;
    r.maps_off = mo;
    r.maps_bytes = maps;
    s->map_builds++;
    return DSDP_OK;
}

void finish(dsdp_sched s, Request *q, int state)
{
    if (q->state == kRunning) {
        s->slots.release(q->slot0, (size_t)q->n_chains);
        s->mem.release(q->arena_off, q->arena_bytes);
        s->receptors[(size_t)q->receptor].active--;
    }
    q->state = state;
    q->t_done = now_s() - s->t0;
    s->finished.push_back(q->ticket);
}

// Admit queued requests in arrival order when their slots, arena space and maps
// fit.  A request that does not fit lets later ones pass, but only for
// kMaxPassedOver rounds: after that nothing behind it is admitted until it is,
// so a request for a receptor whose maps cannot be made resident yet is not
// starved by a stream of requests for resident receptors.
constexpr int kMaxPassedOver = 16;

dsdp_status admit(dsdp_sched s)
{
    bool blocked = false;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request *q = *it;
        if (q->cancel) {
            finish(s, q, kCancelled);
            it = s->queue.erase(it);
            continue;
        }
        if (blocked) break;
        size_t so = 0, ao = 0;
        const size_t ab = align256(q->pl.blob.size() * 4);
        bool ok = s->slots.alloc((size_t)q->n_chains, so);
        if (ok && !s->mem.alloc(ab, ao)) {
            s->slots.release(so, (size_t)q->n_chains);
            ok = false;
        }
        dsdp_status st = DSDP_OK;
        if (ok) {
            st = ensure_resident(s, q->receptor);
            if (st) {
                s->slots.release(so, (size_t)q->n_chains);
                s->mem.release(ao, ab);
                if (st != DSDP_ERR_BUSY) return st;
                ok = false;
            }
        }
        if (!ok) {
            if (++q->passed_over > kMaxPassedOver) blocked = true;
            ++it;
            continue;
        }
        if (st) {
            s->slots.release(so, (size_t)q->n_chains);
            s->mem.release(ao, ab);
            return st;
        }
        HIP_TRY(hipMemcpyAsync(s->pool + ao, q->pl.blob.data(), q->pl.blob.size() * 4, hipMemcpyHostToDevice, s->stream),
                "ligand upload");
        q->slot0 = so;
        q->arena_off = ao;
        q->arena_bytes = ab;
        q->state = kRunning;
        q->fresh = true;
        q->steps_done = 0;
        q->t_admit = now_s() - s->t0;
        Receptor &r = s->receptors[(size_t)q->receptor];
        r.active++;
        r.last_use = ++s->clock;
        s->running.push_back(q);
        it = s->queue.erase(it);
    }
    // blobs are uploaded from request-owned host memory, which outlives the copy
    return DSDP_OK;
}

}  // namespace

extern "C" {

size_t dsdp_sched_fixed_bytes(int32_t slot_capacity)
{
    if (slot_capacity < 1) return 0;
    return fixed_bytes(slot_capacity);
}

dsdp_status dsdp_sched_create(void *d_pool, size_t pool_bytes, int32_t slot_capacity, int32_t steps_per_tick,
                              const dsdp_params *prm, void *stream, dsdp_sched *out)
{
    if (!out) return fail(DSDP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (slot_capacity < 1 || slot_capacity > (1 << 22))
        return fail(DSDP_ERR_INVALID_ARG, "slot_capacity %d outside 1..2^22", slot_capacity);
    if (steps_per_tick < 1) return fail(DSDP_ERR_INVALID_ARG, "steps_per_tick must be >= 1");
    dsdp_status st = check_params(prm);
    if (st) return st;
    if (!d_pool || !aligned256(d_pool)) return fail(DSDP_ERR_INVALID_ARG, "pool must be a 256-byte aligned device buffer");
    if (pool_bytes > ((size_t)1 << 34))
        return fail(DSDP_ERR_UNSUPPORTED, "pool of %zu bytes: at most 16 GiB (ligand offsets are 32-bit words)", pool_bytes);
    const size_t fixed = fixed_bytes(slot_capacity);
    if (pool_bytes < fixed) return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "pool needs at least %zu bytes", fixed);
    std::unique_ptr<dsdp_sched_s> s(new dsdp_sched_s());
    s->pool = (char *)d_pool;
    s->pool_bytes = pool_bytes;
    s->stream = (hipStream_t)stream;
    s->capacity = slot_capacity;
    s->spt = steps_per_tick;
    if (prm)
        s->prm = *prm;
    else
        dsdp_params_default(&s->prm);
    s->sp = to_search(&s->prm);
    size_t o = 0;
    s->off_tasks = o; o += align256((size_t)slot_capacity * sizeof(ChainTask));
    s->off_state = o; o += align256((size_t)slot_capacity * kStWords * 4);
    s->off_records = o; o += align256((size_t)slot_capacity * kRecWords * 4);
    s->off_xyz = o; o += align256((size_t)slot_capacity * kXyzStride * 16);
    s->off_segs = o; o += align256((size_t)slot_capacity * sizeof(RankSeg));
    s->off_sel = o; o += align256((size_t)slot_capacity * 2 * 4);
    s->off_grids = o; o += align256((size_t)kMaxReceptors * sizeof(GridView));
    // the allocator hands out pool offsets in [o, pool_bytes)
    s->mem.init(pool_bytes - o);
    s->mem.free_.clear();
    if (pool_bytes > o) s->mem.free_[o] = pool_bytes - o;
    s->slots.init((size_t)slot_capacity);
    s->h_grids.assign(kMaxReceptors, GridView{});
    s->t0 = now_s();
    *out = s.release();
    return DSDP_OK;
}

void dsdp_sched_destroy(dsdp_sched s) { delete s; }

dsdp_status dsdp_sched_add_receptor(dsdp_sched s, const dsdp_atom *rec, int32_t n_rec, const dsdp_box *box,
                                    const int32_t *types, int32_t n_types, int32_t *receptor_id)
{
    if (!s || !receptor_id) return fail(DSDP_ERR_INVALID_ARG, "scheduler or receptor_id is NULL");
    if ((int)s->receptors.size() >= kMaxReceptors) return fail(DSDP_ERR_UNSUPPORTED, "more than %d receptors", kMaxReceptors);
    int32_t n[3];
    float origin[3];
    dsdp_status st = dsdp_grid_dims(box, n, origin);
    if (st) return st;
    if (n_rec < 0 || (n_rec > 0 && !rec)) return fail(DSDP_ERR_INVALID_ARG, "bad receptor array");
    Receptor r;
    r.atoms.assign(rec, rec + n_rec);
    r.box = *box;
    if (types) {
        if (n_types < 1 || n_types > kNXS) return fail(DSDP_ERR_INVALID_ARG, "n_types %d outside 1..17", n_types);
        r.types.assign(types, types + n_types);
    } else {
        for (int t = 0; t < kNXS; t++) r.types.push_back(t);
    }
    for (int t = 0; t < kNXS; t++) r.map_of_type[t] = -1;
    for (size_t t = 0; t < r.types.size(); t++) {
        const int x = r.types[t];
        if (x < 0 || x >= kNXS || r.map_of_type[x] >= 0) return fail(DSDP_ERR_INVALID_ARG, "bad map type list");
        r.map_of_type[x] = (int)t;
    }
    const size_t maps = align256(dsdp_grids_bytes(box, (int32_t)r.types.size()));
    const size_t wsb = align256(dsdp_build_grids_workspace_bytes(n_rec, box));
    if (maps + wsb > s->mem.total)
        return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "receptor maps need %zu bytes, the pool has %zu", maps + wsb,
                    s->mem.total);
    s->receptors.push_back(std::move(r));
    *receptor_id = (int32_t)s->receptors.size() - 1;
    return DSDP_OK;
}

dsdp_status dsdp_sched_set_site(dsdp_sched s, int32_t receptor_id, const float *points, int32_t n_points,
                                float radius)
{
    if (!s) return fail(DSDP_ERR_INVALID_ARG, "scheduler is NULL");
    if (receptor_id < 0 || receptor_id >= (int)s->receptors.size())
        return fail(DSDP_ERR_INVALID_ARG, "unknown receptor %d", receptor_id);
    if (n_points < 0 || n_points > kMaxSite) return fail(DSDP_ERR_INVALID_ARG, "n_points %d outside 0..%d", n_points, kMaxSite);
    if (n_points > 0 && (!points || !(radius > 0.f) || !std::isfinite(radius)))
        return fail(DSDP_ERR_INVALID_ARG, "site points missing or radius not positive");
    std::vector<float4> site((size_t)n_points);
    for (int i = 0; i < n_points; i++) {
        const float x = points[3 * i], y = points[3 * i + 1], z = points[3 * i + 2];
        if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
            return fail(DSDP_ERR_INVALID_ARG, "site point %d is not finite", i);
        site[(size_t)i] = make_float4(x, y, z, 0.f);
    }
    Receptor &r = s->receptors[(size_t)receptor_id];
    // a running request keeps the search space it started with: change it only
    // while none of this receptor's requests is queued or running
    if (r.active > 0) return fail(DSDP_ERR_BUSY, "receptor %d has running requests", receptor_id);
    for (const Request *q : s->queue)
        if (q->receptor == receptor_id) return fail(DSDP_ERR_BUSY, "receptor %d has queued requests", receptor_id);
    const size_t need = align256(dsdp_grids_bytes(&r.box, (int32_t)r.types.size())) +
                        align256(site.size() * sizeof(float4)) +
                        align256(dsdp_build_grids_workspace_bytes((int32_t)r.atoms.size(), &r.box));
    if (need > s->mem.total)
        return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "receptor maps and site need %zu bytes, the pool has %zu", need,
                    s->mem.total);
    // resident maps are rebuilt with the new points when next needed
    if (r.resident) evict(s, r);
    r.site.swap(site);
    r.site_r = n_points ? radius : 0.f;
    return DSDP_OK;
}

dsdp_status dsdp_sched_submit(dsdp_sched s, int32_t receptor_id, const dsdp_ligand *lig, int32_t n_chains,
                              int32_t n_steps, uint64_t seed, int32_t top_k, int64_t *ticket)
{
    if (!s || !ticket) return fail(DSDP_ERR_INVALID_ARG, "scheduler or ticket is NULL");
    if (receptor_id < 0 || receptor_id >= (int)s->receptors.size())
        return fail(DSDP_ERR_INVALID_ARG, "unknown receptor %d", receptor_id);
    if (n_chains < 1 || n_chains > s->capacity)
        return fail(DSDP_ERR_INVALID_ARG, "n_chains %d outside 1..slot capacity %d", n_chains, s->capacity);
    if (n_steps < 0) return fail(DSDP_ERR_INVALID_ARG, "n_steps < 0");
    if (top_k < 0 || top_k > n_chains) return fail(DSDP_ERR_INVALID_ARG, "top_k %d outside 0..n_chains", top_k);
    dsdp_status st = check_work(&s->prm, n_steps);
    if (st) return st;
    std::unique_ptr<Request> q(new Request());
    st = prepare_ligand(lig, s->receptors[(size_t)receptor_id].map_of_type, q->pl,
                                    intra_ctx(&s->prm, s->capacity, true));
    if (st) return st;
    if (search_lds_bytes(q->pl.h, 1) > device_max_lds())
        return fail(DSDP_ERR_UNSUPPORTED, "ligand needs %zu bytes of LDS", search_lds_bytes(q->pl.h, 1));
    // an idle scheduler must be able to admit it: its ligand next to its receptor's maps
    const Receptor &r = s->receptors[(size_t)receptor_id];
    const size_t need = align256(q->pl.blob.size() * 4) + align256(dsdp_grids_bytes(&r.box, (int32_t)r.types.size())) +
                        align256(r.site.size() * sizeof(float4)) +
                        align256(dsdp_build_grids_workspace_bytes((int32_t)r.atoms.size(), &r.box));
    if (need > s->mem.total)
        return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "request needs %zu pool bytes, the pool has %zu", need, s->mem.total);
    q->ticket = s->next_ticket++;
    q->receptor = receptor_id;
    q->n_chains = n_chains;
    q->n_steps = n_steps;
    q->seed = seed;
    q->top_k = top_k;
    q->t_submit = now_s() - s->t0;
    *ticket = q->ticket;
    s->queue.push_back(q.get());
    s->requests[q->ticket] = std::move(q);
    return DSDP_OK;
}

dsdp_status dsdp_sched_cancel(dsdp_sched s, int64_t ticket)
{
    if (!s) return fail(DSDP_ERR_INVALID_ARG, "scheduler is NULL");
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return fail(DSDP_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    it->second->cancel = true;
    return DSDP_OK;
}

dsdp_status dsdp_sched_tick(dsdp_sched s, int32_t *n_completed)
{
    if (n_completed) *n_completed = 0;
    if (!s) return fail(DSDP_ERR_INVALID_ARG, "scheduler is NULL");
    // drop cancelled running requests, then admit
    for (auto it = s->running.begin(); it != s->running.end();) {
        if ((*it)->cancel) {
            finish(s, *it, kCancelled);
            it = s->running.erase(it);
        } else {
            ++it;
        }
    }
    dsdp_status st = admit(s);
    if (st) return st;
    if (s->running.empty()) return DSDP_OK;
    s->ticks++;

    // tasks of every running chain, in launch groups (kernel variant and LDS need)
    s->h_tasks.clear();
    std::vector<LaunchGroup> groups;
    {
        std::vector<const LigHeader *> hdr;
        std::vector<long> ch;
        for (Request *q : s->running) {
            hdr.push_back(&q->pl.h);
            ch.push_back(q->n_chains);
        }
        st = plan_groups(&s->prm, hdr, ch, groups);
        if (st) return st;
    }
    std::vector<long> first;
    for (const LaunchGroup &g : groups) {
        first.push_back((long)s->h_tasks.size());
        for (int m : g.members) {
            const Request *q = s->running[(size_t)m];
            for (int c = 0; c < q->n_chains; c++) {
                ChainTask t{};
                t.blob_off = (uint32_t)(q->arena_off / 4);
                t.blob_words = (uint32_t)q->pl.h.total_words;
                t.chain = (uint32_t)c;
                t.n_steps = q->n_steps;
                t.seed_lo = (uint32_t)q->seed;
                t.seed_hi = (uint32_t)(q->seed >> 32);
                t.grid = q->receptor;
                t.slot = (int32_t)(q->slot0 + c);
                t.fresh = q->fresh ? 1 : 0;
                s->h_tasks.push_back(t);
            }
        }
    }
    HIP_TRY(hipMemcpyAsync(s->pool + s->off_tasks, s->h_tasks.data(), s->h_tasks.size() * sizeof(ChainTask),
                           hipMemcpyHostToDevice, s->stream),
            "task upload");
    if (s->grids_dirty) {
        HIP_TRY(hipMemcpyAsync(s->pool + s->off_grids, s->h_grids.data(), s->h_grids.size() * sizeof(GridView),
                               hipMemcpyHostToDevice, s->stream),
                "grid upload");
        s->grids_dirty = false;
    }
    for (size_t k = 0; k < groups.size(); k++) {
        const LaunchGroup &g = groups[k];
        HIP_TRY(launch_tick(g.cls, g.waves, g.lds, (const uint32_t *)s->pool,
                            (const ChainTask *)(s->pool + s->off_tasks) + first[k], (int)g.chains,
                            (const GridView *)(s->pool + s->off_grids), s->sp, s->spt, 0,
                            (float *)(s->pool + s->off_state), (float *)(s->pool + s->off_records),
                            (float4 *)(s->pool + s->off_xyz), s->stream),
                "tick launch");
    }
    // requests whose chains finish in this tick
    std::vector<Request *> done;
    for (Request *q : s->running) {
        q->fresh = false;
        q->steps_done = std::min(q->n_steps, q->steps_done + s->spt);
        if (q->steps_done >= q->n_steps) done.push_back(q);
    }
    std::vector<std::vector<float>> recs(done.size());
    std::vector<int> h_sel;
    if (!done.empty()) {
        s->h_segs.clear();
        int sel_off = 0, max_chains = 1;
        for (Request *q : done) {
            RankSeg g;
            g.slot0 = (int32_t)q->slot0;
            g.n_chains = q->n_chains;
            g.n_atoms = q->pl.h.n_atoms;
            g.top_k = q->top_k;
            g.sel_off = sel_off;
            sel_off += q->n_chains + 1;
            max_chains = std::max(max_chains, q->n_chains);
            s->h_segs.push_back(g);
        }
        HIP_TRY(hipMemcpyAsync(s->pool + s->off_segs, s->h_segs.data(), s->h_segs.size() * sizeof(RankSeg),
                               hipMemcpyHostToDevice, s->stream),
                "segment upload");
        HIP_TRY(launch_rank((const float *)(s->pool + s->off_records), (const float4 *)(s->pool + s->off_xyz),
                            (const RankSeg *)(s->pool + s->off_segs), (int)done.size(), max_chains,
                            s->sp.rmsd_cluster, (int *)(s->pool + s->off_sel), s->stream),
                "rank launch");
        h_sel.resize((size_t)sel_off);
        HIP_TRY(hipMemcpyAsync(h_sel.data(), s->pool + s->off_sel, h_sel.size() * 4, hipMemcpyDeviceToHost, s->stream),
                "result copy");
        for (size_t k = 0; k < done.size(); k++) {
            Request *q = done[k];
            recs[k].resize((size_t)q->n_chains * kRecWords);
            HIP_TRY(hipMemcpyAsync(recs[k].data(), s->pool + s->off_records + q->slot0 * kRecWords * 4,
                                   recs[k].size() * 4, hipMemcpyDeviceToHost, s->stream),
                    "result copy");
        }
    }
    HIP_TRY(hipStreamSynchronize(s->stream), "tick");
    for (size_t k = 0; k < done.size(); k++) {
        Request *q = done[k];
        const int *sl = &h_sel[(size_t)s->h_segs[k].sel_off];
        const int cnt = q->top_k > 0 ? sl[0] : 0;
        q->result.resize((size_t)cnt);
        for (int r = 0; r < cnt; r++) fill_pose(&recs[k][(size_t)sl[1 + r] * kRecWords], q->pl.h.n_tors, sl[1 + r], q->result[(size_t)r]);
        std::memset(&q->stats, 0, sizeof q->stats);
        add_stats(recs[k].data(), q->n_chains, &q->stats);
        finish(s, q, kDone);
        s->running.erase(std::find(s->running.begin(), s->running.end(), q));
        s->completed++;
    }
    if (n_completed) *n_completed = (int32_t)done.size();
    return DSDP_OK;
}

dsdp_status dsdp_sched_poll(dsdp_sched s, int64_t ticket, int32_t *state, dsdp_pose *out, int32_t *n_out,
                            double *times, dsdp_dock_stats *stats)
{
    if (!s || !state) return fail(DSDP_ERR_INVALID_ARG, "scheduler or state is NULL");
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return fail(DSDP_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    const Request *q = it->second.get();
    *state = q->state;
    if (times) {
        times[0] = q->t_submit;
        times[1] = q->t_admit;
        times[2] = q->t_done;
    }
    if (q->state == kDone) {
        if (out)
            for (size_t r = 0; r < q->result.size(); r++) out[r] = q->result[r];
        if (n_out) *n_out = (int32_t)q->result.size();
        if (stats) *stats = q->stats;
    } else if (n_out) {
        *n_out = 0;
    }
    return DSDP_OK;
}

dsdp_status dsdp_sched_drain(dsdp_sched s, int64_t *tickets, int32_t cap, int32_t *n)
{
    if (!s || !n || (cap > 0 && !tickets)) return fail(DSDP_ERR_INVALID_ARG, "scheduler, tickets or n is NULL");
    int32_t k = 0;
    while (k < cap && !s->finished.empty()) {
        tickets[k++] = s->finished.front();
        s->finished.pop_front();
    }
    *n = k;
    return DSDP_OK;
}

dsdp_status dsdp_sched_release(dsdp_sched s, int64_t ticket)
{
    if (!s) return fail(DSDP_ERR_INVALID_ARG, "scheduler is NULL");
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return fail(DSDP_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    if (it->second->state != kDone && it->second->state != kCancelled)
        return fail(DSDP_ERR_BUSY, "ticket %lld is still queued or running", (long long)ticket);
    s->requests.erase(it);
    return DSDP_OK;
}

dsdp_status dsdp_sched_get_info(dsdp_sched s, dsdp_sched_info *info)
{
    if (!s || !info) return fail(DSDP_ERR_INVALID_ARG, "scheduler or info is NULL");
    std::memset(info, 0, sizeof *info);
    info->queued = (int32_t)s->queue.size();
    info->running = (int32_t)s->running.size();
    info->completed = s->completed;
    for (const Receptor &r : s->receptors) info->resident_receptors += r.resident ? 1 : 0;
    info->free_slots = (int32_t)(s->slots.total - s->slots.used);
    info->pool_bytes = (int64_t)s->pool_bytes;
    info->pool_free = (int64_t)(s->mem.total - s->mem.used);
    info->map_builds = s->map_builds;
    info->evictions = s->evictions;
    info->ticks = s->ticks;
    return DSDP_OK;
}

}  // extern "C"
