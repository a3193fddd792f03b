// Pools: many independent domains advanced together by one launch per kernel per step, with
// the step loop captured once per chunk as a HIP graph. Contracts: include/lbm.h.
#include <cstring>
#include <new>

#include "lbm_domain.h"

using namespace lbm;

struct lbm_pool {
    int32_t precision = LBM_FP64;
    int32_t max_slots = 0;
    int32_t chunk = 100;
    int64_t budget = 0, used = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<lbm_domain*> slots;
    int64_t step = 0;
    int32_t grid = 0, default_grid = 0, cus = 1;
    int32_t order = 1;                // 0: linear tile order, 1: XCD-aware runs

    // Device tables of the batched kernels (fixed addresses, so captured graphs stay valid).
    StepArgs* d_doms = nullptr;
    int32_t* d_tile_first = nullptr;
    int32_t* d_tile_dom = nullptr;
    int32_t* d_ntiles = nullptr;
    int64_t tile_cap = 0;
    double* d_partials = nullptr;
    double* d_red = nullptr;
    std::vector<StepArgs> h_doms;
    std::vector<int32_t> h_tile_first, h_tile_dom;
    std::vector<int32_t> h_group_first, h_group_ntiles;
    int32_t h_ntiles = 0;
    int32_t lookup = LBM_NBR_TABLE;   // the members' common neighbour lookup, else AUTO (mixed)
    bool dirty = true;

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t replays = 0, eager = 0;

    // Device memory of the pool's own tables: the caller's hook, else hipMalloc.
    lbm_allocator alloc{};
    bool has_alloc = false;
    hipError_t dmalloc(void** out, size_t bytes) {
        bytes = std::max<size_t>(bytes, 256);
        if (!has_alloc) return hipMalloc(out, bytes);
        *out = alloc.alloc(bytes, alloc.ctx);
        return *out ? hipSuccess : hipErrorOutOfMemory;
    }
    void dfree(void* ptr) {
        if (!ptr) return;
        if (has_alloc)
            alloc.free(ptr, alloc.ctx);
        else
            (void)hipFree(ptr);
    }

    // Cache groups of the captured chunk (group_bytes > 0): consecutive members whose device
    // footprints sum to at most group_bytes run the whole chunk before the next group starts,
    // so a group's state can stay in the last-level cache across its steps. Group g covers
    // tiles [first, first + ntiles) of the tile table; its launches see that range through
    // d_group_ntiles[g] and a tile_first table relative to its first tile (d_group_first,
    // max_slots entries per group).
    struct Group {
        int32_t first = 0, ntiles = 0;
        std::vector<int32_t> members, offsets;   // slots, and their first tiles - first
        bool operator==(const Group& o) const {
            return first == o.first && ntiles == o.ntiles && members == o.members &&
                   offsets == o.offsets;
        }
    };
    int64_t group_bytes = 0;
    std::vector<Group> groups;
    int32_t* d_group_first = nullptr;
    int32_t* d_group_ntiles = nullptr;
    size_t group_cap = 0;             // groups the two device arrays hold

    BatchArgs batch() const {
        return BatchArgs{d_doms, d_tile_dom, d_tile_first, d_ntiles, order};
    }
    BatchArgs group_batch(size_t g) const {
        return BatchArgs{d_doms, d_tile_dom + groups[g].first,
                         d_group_first + g * (size_t)max_slots, d_group_ntiles + g, order};
    }
    // Workgroups of the batched launch: the XCD-aware order needs whole runs on every XCD.
    int32_t launch_grid() const {
        const int32_t g = 8 * kXcdRun;
        return order ? (grid + g - 1) / g * g : grid;
    }

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

namespace lbm {
// A member's parameters changed (lbm_set_force): the batched kernels read them from the slot
// table, which is uploaded again before the next step. A member with pressure faces also has
// boundary launches of its own in the captured chunk, and those carry its arguments by value
// (the flux inlet's body force), so the chunk is captured again.
lbm_status pool_member_changed(lbm_pool* p, const lbm_domain* d) {
    p->dirty = true;
    if (d->p.bc_z == 1) {
        HIP_TRY(hipStreamSynchronize(p->stream));
        p->drop_graph();
    }
    return LBM_OK;
}
}  // namespace lbm

namespace {

constexpr int kPoolBlock = 256;  // voxels per tile = threads per workgroup

int32_t highest_slot(const lbm_pool* p) {
    int32_t n = 0;
    for (int32_t s = 0; s < p->max_slots; ++s)
        if (p->slots[s]) n = s + 1;
    return n;
}

// Cache groups (see lbm_pool::Group): members in slot order, a new group whenever the next
// member would take the group past group_bytes. A change of the grouping invalidates the
// captured chunk. Uploads are asynchronous on the pool's stream; the caller synchronises.
lbm_status upload_groups(lbm_pool* p) {
    std::vector<lbm_pool::Group> groups;
    if (p->group_bytes > 0) {
        int64_t bytes = 0;
        for (int32_t s = 0; s < p->max_slots; ++s) {
            lbm_domain* d = p->slots[s];
            if (!d) continue;
            const int32_t nt = (int32_t)((d->pre.n_pore + kPoolBlock - 1) / kPoolBlock);
            if (groups.empty() || bytes + d->device_bytes > p->group_bytes) {
                groups.emplace_back();
                groups.back().first = p->h_tile_first[s];
                bytes = 0;
            }
            groups.back().ntiles += nt;
            groups.back().members.push_back(s);
            groups.back().offsets.push_back(p->h_tile_first[s] - groups.back().first);
            bytes += d->device_bytes;
        }
    }
    if (groups == p->groups && (groups.empty() || p->group_cap >= groups.size())) return LBM_OK;
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->drop_graph();
    if (groups.size() > p->group_cap) {
        const size_t cap = std::max(groups.size(), 2 * p->group_cap);
        int32_t *first = nullptr, *nt = nullptr;
        if (p->dmalloc((void**)&first, sizeof(int32_t) * cap * p->max_slots) != hipSuccess ||
            p->dmalloc((void**)&nt, sizeof(int32_t) * cap) != hipSuccess) {
            p->dfree(first);
            return fail(LBM_ERR_OOM, "device allocation failed (pool groups)");
        }
        p->dfree(p->d_group_first);
        p->dfree(p->d_group_ntiles);
        p->d_group_first = first;
        p->d_group_ntiles = nt;
        p->group_cap = cap;
    }
    p->groups = groups;
    if (groups.empty()) return LBM_OK;
    p->h_group_first.assign(groups.size() * (size_t)p->max_slots, 0);
    p->h_group_ntiles.assign(groups.size(), 0);
    for (size_t g = 0; g < groups.size(); ++g) {
        p->h_group_ntiles[g] = groups[g].ntiles;
        for (size_t k = 0; k < groups[g].members.size(); ++k)
            p->h_group_first[g * p->max_slots + groups[g].members[k]] = groups[g].offsets[k];
    }
    HIP_TRY(hipMemcpyAsync(p->d_group_first, p->h_group_first.data(),
                           sizeof(int32_t) * p->h_group_first.size(), hipMemcpyHostToDevice,
                           p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_group_ntiles, p->h_group_ntiles.data(),
                           sizeof(int32_t) * p->h_group_ntiles.size(), hipMemcpyHostToDevice,
                           p->stream));
    return LBM_OK;
}

// Rebuild and upload the per-slot arguments and the tile table after a membership change.
lbm_status upload_tables(lbm_pool* p) {
    p->h_doms.assign(p->max_slots, StepArgs{});
    p->h_tile_first.assign(p->max_slots, 0);
    p->h_tile_dom.clear();
    for (int32_t s = 0; s < p->max_slots; ++s) {
        lbm_domain* d = p->slots[s];
        p->h_tile_first[s] = (int32_t)p->h_tile_dom.size();
        if (!d) continue;
        p->h_doms[s] = d->args(kPoolBlock, 1);
        const int64_t nt = (d->pre.n_pore + kPoolBlock - 1) / kPoolBlock;
        p->h_tile_dom.insert(p->h_tile_dom.end(), (size_t)nt, s);
    }
    p->h_ntiles = (int32_t)p->h_tile_dom.size();
    // The step kernels are specialised on the neighbour lookup when all members share it; a
    // change of that choice invalidates the captured graph.
    int n_rank = 0, n_compact = 0, n_members = 0;
    for (lbm_domain* d : p->slots)
        if (d) {
            ++n_members;
            n_rank += d->rank ? 1 : 0;
            n_compact += d->compact ? 1 : 0;
        }
    const int32_t lookup = n_rank == n_members && n_members ? LBM_NBR_RANK
                           : n_compact == n_members && n_members ? LBM_NBR_COMPACT
                           : n_rank == 0 && n_compact == 0 ? LBM_NBR_TABLE : LBM_NBR_AUTO;
    if (lookup != p->lookup) {
        HIP_TRY(hipStreamSynchronize(p->stream));
        p->drop_graph();
        p->lookup = lookup;
    }
    if ((int64_t)p->h_tile_dom.size() > p->tile_cap) {
        // Grow the tile table; its address is baked into the captured graph.
        int64_t cap = std::max<int64_t>(p->tile_cap * 2, (int64_t)p->h_tile_dom.size());
        int32_t* ptr = nullptr;
        HIP_TRY(hipStreamSynchronize(p->stream));
        if (p->dmalloc((void**)&ptr, sizeof(int32_t) * cap) != hipSuccess)
            return fail(LBM_ERR_OOM, "device allocation failed (pool tile table)");
        p->dfree(p->d_tile_dom);
        p->d_tile_dom = ptr;
        p->tile_cap = cap;
        p->drop_graph();
    }
    HIP_TRY(hipMemcpyAsync(p->d_doms, p->h_doms.data(), sizeof(StepArgs) * p->max_slots,
                           hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_tile_first, p->h_tile_first.data(),
                           sizeof(int32_t) * p->max_slots, hipMemcpyHostToDevice, p->stream));
    if (p->h_ntiles)
        HIP_TRY(hipMemcpyAsync(p->d_tile_dom, p->h_tile_dom.data(),
                               sizeof(int32_t) * p->h_ntiles, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_ntiles, &p->h_ntiles, sizeof(int32_t), hipMemcpyHostToDevice,
                           p->stream));
    if (lbm_status st = upload_groups(p)) return st;
    // The host vectors stay alive and unchanged until the next upload, which first waits for
    // the stream, so the asynchronous copies never read a buffer being rewritten.
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->dirty = false;
    return LBM_OK;
}

// A member with pressure faces gets the boundary work of its single-domain step between and
// after the batched launches, in the same order: the ghost phi entries after the phase kernel,
// then (flux inlet) the inlet density and the pressure faces after the collide kernel.
lbm_status launch_face_work(lbm_pool* p, const std::vector<int32_t>& members, bool odd,
                            bool after_collide) {
    for (int32_t s : members) {
        lbm_domain* d = p->slots[s];
        if (!d || d->p.bc_z != 1) continue;
        const StepArgs a = d->args();
        if (!after_collide) {
            if (!d->rank && !d->pre.ghost_tail.empty())
                HIP_TRY(launch_ghosts(a, d->ghost_tail, d->ghost_src,
                                      (int32_t)d->pre.ghost_tail.size(), p->stream));
            continue;
        }
        // The member's reduction partials are free between reductions: scratch for the inlet.
        if (d->inlet_rho)
            HIP_TRY(launch_inlet_density(a, !odd, d->faces, (int32_t)d->pre.inlet.size(),
                                         d->p.flux_in, d->inlet_rho, d->red_partials,
                                         p->stream));
        HIP_TRY(launch_pressure_bc(a, !odd, d->faces, (int32_t)d->pre.inlet.size(),
                                   (int32_t)d->pre.outlet.size(), d->p.rho_in, d->p.rho_out,
                                   d->inlet_rho, p->stream));
    }
    return LBM_OK;
}

// n steps of the members in `members` over the tiles that b covers.
lbm_status launch_steps_of(lbm_pool* p, const BatchArgs& b, const std::vector<int32_t>& members,
                           int64_t first_step, int64_t n) {
    for (int64_t k = 0; k < n; ++k) {
        const bool odd = ((first_step + k) & 1) != 0;
        HIP_TRY(launch_phase_batched(b, p->precision, odd, p->lookup, p->launch_grid(),
                                     kPoolBlock, p->stream));
        if (lbm_status st = launch_face_work(p, members, odd, false)) return st;
        HIP_TRY(launch_collide_batched(b, p->precision, odd, p->lookup, p->launch_grid(),
                                       kPoolBlock, p->stream));
        if (lbm_status st = launch_face_work(p, members, odd, true)) return st;
    }
    return LBM_OK;
}

std::vector<int32_t> all_members(const lbm_pool* p) {
    std::vector<int32_t> m;
    for (int32_t s = 0; s < p->max_slots; ++s)
        if (p->slots[s]) m.push_back(s);
    return m;
}

// n steps of every member, each step one batched launch per kernel over all tiles.
lbm_status launch_steps(lbm_pool* p, int64_t first_step, int64_t n) {
    return launch_steps_of(p, p->batch(), all_members(p), first_step, n);
}

lbm_status capture(lbm_pool* p) {
    p->drop_graph();
    HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    // Chunks start on even steps. With cache groups, each group takes the whole chunk in turn
    // (members are independent, so only the order of their launches changes).
    lbm_status st = LBM_OK;
    if (p->groups.empty()) {
        st = launch_steps(p, 0, p->chunk);
    } else {
        for (size_t g = 0; g < p->groups.size() && st == LBM_OK; ++g) {
            const std::vector<int32_t>& members = p->groups[g].members;
            if (members.size() == 1) {
                // A member alone in its group gains nothing from the batched launch: its chunk
                // runs the single-domain launches with the member's own configuration (for a
                // large member, streaming accesses and workgroup limits). Same arithmetic per
                // voxel, so the result is the same bitwise.
                lbm_domain* d = p->slots[members[0]];
                for (int64_t k = 0; k < p->chunk && st == LBM_OK; ++k)
                    st = launch_domain_step(d, (k & 1) != 0);
            } else {
                st = launch_steps_of(p, p->group_batch(g), members, 0, p->chunk);
            }
        }
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->stream, &g);
    if (st != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    p->graph = g;
    HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return LBM_OK;
}

void advance_members(lbm_pool* p, int64_t n) {
    for (lbm_domain* d : p->slots)
        if (d) d->step += n;
    p->step += n;
}

}  // namespace

extern "C" {

lbm_status lbm_pool_create(int64_t hbm_budget_bytes, int32_t precision, int32_t max_slots,
                           int32_t chunk_steps, const lbm_allocator* alloc, void* hip_stream,
                           lbm_pool** out) {
    if (!out) return fail(LBM_ERR_ARG, "out must be non-null");
    *out = nullptr;
    if (hbm_budget_bytes <= 0 || max_slots <= 0 || max_slots > 4096)
        return fail(LBM_ERR_ARG, "need hbm_budget_bytes > 0 and 0 < max_slots <= 4096");
    if (precision != LBM_FP64 && precision != LBM_FP32_DEV && precision != LBM_FP32_MIXED)
        return fail(LBM_ERR_ARG, "precision must be a lbm_precision");
    if (chunk_steps < 2 || (chunk_steps & 1)) return fail(LBM_ERR_ARG, "chunk_steps must be even and >= 2");
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(LBM_ERR_ARG, "allocator needs both alloc and free");
    lbm_pool* p = new (std::nothrow) lbm_pool();
    if (!p) return fail(LBM_ERR_OOM, "host allocation failed");
    if (alloc) {
        p->alloc = *alloc;
        p->has_alloc = true;
    }
    p->precision = precision;
    p->max_slots = max_slots;
    p->chunk = chunk_steps;
    p->budget = hbm_budget_bytes;
    p->slots.assign(max_slots, nullptr);
    auto bail = [&](lbm_status s, const std::string& m) {
        lbm_pool_destroy(p);
        return fail(s, m);
    };
    if (hip_stream) {
        p->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(LBM_ERR_DEVICE, "stream creation failed");
        p->own_stream = true;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return bail(LBM_ERR_DEVICE, "device query failed");
    // Defaults: 32 workgroups per compute unit in the XCD-aware order, what the autotuner picks
    // for uneven batches of 48..160-voxel volumes.
    p->cus = std::max(1, cus);
    p->default_grid = p->grid = p->cus * 32;
    p->tile_cap = 1 << 16;
    if (p->dmalloc((void**)&p->d_doms, sizeof(StepArgs) * max_slots) != hipSuccess ||
        p->dmalloc((void**)&p->d_tile_first, sizeof(int32_t) * max_slots) != hipSuccess ||
        p->dmalloc((void**)&p->d_tile_dom, sizeof(int32_t) * p->tile_cap) != hipSuccess ||
        p->dmalloc((void**)&p->d_ntiles, sizeof(int32_t)) != hipSuccess ||
        p->dmalloc((void**)&p->d_partials,
                   sizeof(double) * kNRed * kRedBlocks * (size_t)max_slots) != hipSuccess ||
        p->dmalloc((void**)&p->d_red, sizeof(double) * kNRed * (size_t)max_slots) != hipSuccess)
        return bail(LBM_ERR_OOM, "device allocation failed");
    if (lbm_status s = upload_tables(p)) {
        lbm_pool_destroy(p);
        return s;
    }
    *out = p;
    return LBM_OK;
}

lbm_status lbm_pool_admit(lbm_pool* p, lbm_domain* d, int32_t* slot) {
    if (!p || !d || !slot) return fail(LBM_ERR_ARG, "null argument");
    if (d->pool) return fail(LBM_ERR_STATE, "the domain already belongs to a pool");
    if (d->p.precision != p->precision) return fail(LBM_ERR_STATE, "precision differs from the pool's");
    if ((d->step & 1) != (p->step & 1))
        return fail(LBM_ERR_STATE, "step parity differs from the pool's");
    if (d->unstable) return fail(LBM_ERR_UNSTABLE, "the domain is unstable");
    if (p->used + d->device_bytes > p->budget) return fail(LBM_ERR_OOM, "HBM budget exhausted");
    int32_t s = -1;
    for (int32_t k = 0; k < p->max_slots && s < 0; ++k)
        if (!p->slots[k]) s = k;
    if (s < 0) return fail(LBM_ERR_OOM, "no free slot");
    HIP_TRY(hipStreamSynchronize(d->stream));
    if (d->p.bc_z == 1) {
        // The captured chunk holds the face work of every member with pressure faces.
        HIP_TRY(hipStreamSynchronize(p->stream));
        p->drop_graph();
    }
    d->own_stream_saved = d->stream;
    d->stream = p->stream;
    d->pool = p;
    p->slots[s] = d;
    p->used += d->device_bytes;
    p->dirty = true;
    *slot = s;
    return LBM_OK;
}

lbm_status lbm_pool_retire(lbm_pool* p, int32_t slot, lbm_domain** out) {
    if (out) *out = nullptr;
    if (!p || slot < 0 || slot >= p->max_slots || !p->slots[slot])
        return fail(LBM_ERR_ARG, "no member in that slot");
    lbm_domain* d = p->slots[slot];
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (d->p.bc_z == 1) p->drop_graph();
    d->stream = d->own_stream_saved;
    d->own_stream_saved = nullptr;
    d->pool = nullptr;
    p->slots[slot] = nullptr;
    p->used -= d->device_bytes;
    p->dirty = true;
    if (out) *out = d;
    return LBM_OK;
}

lbm_status lbm_pool_step(lbm_pool* p, int64_t nsteps) {
    if (!p) return fail(LBM_ERR_ARG, "null pool");
    if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
    for (lbm_domain* d : p->slots)
        if (d && d->unstable) return fail(LBM_ERR_UNSTABLE, "a member is unstable; retire it");
    if (p->dirty)
        if (lbm_status s = upload_tables(p)) return s;
    int64_t left = nsteps;
    while (left > 0) {
        if (p->h_ntiles == 0) {             // no members: only the step count moves
            advance_members(p, left);
            break;
        }
        if (left >= p->chunk && (p->step & 1) == 0) {
            if (!p->exec)
                if (lbm_status s = capture(p)) return s;
            HIP_TRY(hipGraphLaunch(p->exec, p->stream));
            ++p->replays;
            advance_members(p, p->chunk);
            left -= p->chunk;
        } else {
            if (lbm_status s = launch_steps(p, p->step, 1)) return s;
            ++p->eager;
            advance_members(p, 1);
            left -= 1;
        }
    }
    return LBM_OK;
}

lbm_status lbm_pool_reduce(lbm_pool* p, int32_t slot, lbm_reduction* out) {
    if (!p || !out) return fail(LBM_ERR_ARG, "null argument");
    if (slot < 0 || slot >= p->max_slots || !p->slots[slot])
        return fail(LBM_ERR_ARG, "no member in that slot");
    // A member runs on the pool's stream; its own reduction is the single-domain one, whose
    // decomposition the batched reduction reproduces bit for bit.
    return lbm_reduce(p->slots[slot], out);
}

lbm_status lbm_pool_reduce_all(lbm_pool* p, lbm_reduction* out, int32_t max_count,
                               int32_t* count) {
    if (!p || !count || (max_count > 0 && !out)) return fail(LBM_ERR_ARG, "null argument");
    if (p->dirty)
        if (lbm_status s = upload_tables(p)) return s;
    const int32_t n = std::min(highest_slot(p), std::max(max_count, 0));
    std::vector<double> acc((size_t)std::max(n, 1) * kNRed);
    if (n > 0) {
        HIP_TRY(launch_reduce_batched(p->batch(), p->precision, (p->step & 1) != 0, n,
                                      p->d_partials, p->d_red, p->stream));
        HIP_TRY(hipMemcpyAsync(acc.data(), p->d_red, sizeof(double) * kNRed * n,
                               hipMemcpyDeviceToHost, p->stream));
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    for (int32_t s = 0; s < n; ++s) {
        if (p->slots[s]) {
            finish_reduction(p->slots[s], &acc[(size_t)s * kNRed], p->slots[s]->step, &out[s]);
            if (out[s].unstable) p->slots[s]->unstable = true;
        } else {
            std::memset(&out[s], 0, sizeof out[s]);
        }
    }
    *count = n;
    return LBM_OK;
}

lbm_status lbm_pool_get_info(lbm_pool* p, lbm_pool_info* out) {
    if (!p || !out) return fail(LBM_ERR_ARG, "null argument");
    std::memset(out, 0, sizeof *out);
    out->max_slots = p->max_slots;
    for (lbm_domain* d : p->slots) out->members += d ? 1 : 0;
    out->chunk_steps = p->chunk;
    out->grid = p->grid;
    out->step = p->step;
    out->used_bytes = p->used;
    out->budget_bytes = p->budget;
    out->tiles = p->dirty ? -1 : p->h_ntiles;
    out->graph_replays = p->replays;
    out->eager_steps = p->eager;
    out->order = p->order;
    out->groups = p->dirty ? -1 : (int32_t)p->groups.size();
    return LBM_OK;
}

lbm_status lbm_pool_set_order(lbm_pool* p, int32_t order) {
    if (!p || (order != 0 && order != 1)) return fail(LBM_ERR_ARG, "order must be 0 or 1");
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->order = order;
    p->drop_graph();
    return LBM_OK;
}

lbm_status lbm_pool_set_group_bytes(lbm_pool* p, int64_t group_bytes) {
    if (!p || group_bytes < 0) return fail(LBM_ERR_ARG, "group_bytes must be >= 0");
    p->group_bytes = group_bytes;
    p->dirty = true;
    return LBM_OK;
}

lbm_status lbm_pool_set_grid(lbm_pool* p, int32_t grid) {
    if (!p || grid < 0 || grid > (1 << 20)) return fail(LBM_ERR_ARG, "bad grid");
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->grid = grid ? grid : p->default_grid;
    p->drop_graph();
    return LBM_OK;
}

lbm_status lbm_pool_autotune(lbm_pool* p, int32_t trial_steps, int32_t* grid) {
    if (!p) return fail(LBM_ERR_ARG, "null pool");
    if (trial_steps < 2) return fail(LBM_ERR_ARG, "trial_steps must be >= 2");
    trial_steps += trial_steps & 1;
    if (p->dirty)
        if (lbm_status s = upload_tables(p)) return s;
    // Snapshot every member's populations (device to device).
    struct Snap { lbm_domain* d; void* buf; size_t bytes; };
    std::vector<Snap> snaps;
    lbm_status st = LBM_OK;
    for (lbm_domain* d : p->slots) {
        if (!d) continue;
        const size_t fb = d->f_bytes(), eb = d->m_bytes(), ld = (size_t)d->pre.ld;
        Snap sn{d, nullptr, (fb * 19 + eb * 8) * ld + sizeof(int32_t)};
        if (p->dmalloc(&sn.buf, sn.bytes) != hipSuccess) {
            st = fail(LBM_ERR_OOM, "no device memory for the autotuner's snapshot");
            break;
        }
        snaps.push_back(sn);
        size_t off = 0;
        void* arr[3] = {d->f, d->M, d->fresh};
        const size_t sizes[3] = {fb * 19 * ld, eb * 8 * ld, sizeof(int32_t)};
        for (int k = 0; k < 3 && st == LBM_OK; ++k) {
            if (hipMemcpyAsync((char*)sn.buf + off, arr[k], sizes[k], hipMemcpyDeviceToDevice,
                               p->stream) != hipSuccess)
                st = fail(LBM_ERR_DEVICE, "snapshot copy failed");
            off += sizes[k];
        }
    }
    const int64_t step0 = p->step;
    std::vector<int64_t> dstep0;
    for (const Snap& sn : snaps) dstep0.push_back(sn.d->step);
    const int32_t keep = p->grid, keep_order = p->order;
    int32_t best = keep, best_order = keep_order;
    double best_ms = 1e30;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == LBM_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(LBM_ERR_DEVICE, "event creation failed");
    const int mult[5] = {2, 4, 8, 16, 32};
    for (int c = 0; c < 10 && st == LBM_OK && p->h_ntiles > 0; ++c) {
        p->grid = p->cus * mult[c % 5];
        p->order = c / 5;
        st = launch_steps(p, p->step, 2);                      // warm-up
        if (st != LBM_OK) break;
        if (hipEventRecord(e0, p->stream) != hipSuccess) { st = fail(LBM_ERR_DEVICE, "event"); break; }
        st = launch_steps(p, p->step + 2, trial_steps);
        if (st != LBM_OK) break;
        float ms = 0.f;
        if (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = fail(LBM_ERR_DEVICE, "event timing failed");
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = p->grid;
            best_order = p->order;
        }
    }
    // Cache groups: with the chosen grid and order, one warm-up and one timed replay of the
    // captured chunk per candidate group size (needs the pool at an even step, like any chunk).
    const int64_t keep_group = p->group_bytes;
    int64_t best_group = keep_group;
    if (st == LBM_OK) {
        p->grid = best;
        p->order = best_order;
        p->drop_graph();
    }
    if (st == LBM_OK && (p->step & 1) == 0 && p->h_ntiles > 0) {
        const int64_t MiB = 1 << 20;
        const int64_t cand[6] = {0, 128 * MiB, 192 * MiB, 256 * MiB, 320 * MiB, 384 * MiB};
        double best_chunk = 1e30;
        for (int c = 0; c < 6 && st == LBM_OK; ++c) {
            p->group_bytes = cand[c];
            if ((st = upload_groups(p)) != LBM_OK) break;
            if (hipStreamSynchronize(p->stream) != hipSuccess) { st = fail(LBM_ERR_DEVICE, "sync"); break; }
            if (!p->exec && (st = capture(p)) != LBM_OK) break;
            float ms = 0.f;
            if (hipGraphLaunch(p->exec, p->stream) != hipSuccess ||
                hipEventRecord(e0, p->stream) != hipSuccess ||
                hipGraphLaunch(p->exec, p->stream) != hipSuccess ||
                hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(LBM_ERR_DEVICE, "chunk timing failed");
                break;
            }
            if (ms < best_chunk) {
                best_chunk = ms;
                best_group = cand[c];
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // Restore states; the trial steps came in even numbers, so parities are unchanged.
    for (size_t k = 0; k < snaps.size(); ++k) {
        lbm_domain* d = snaps[k].d;
        const size_t fb = d->f_bytes(), eb = d->m_bytes(), ld = (size_t)d->pre.ld;
        size_t off = 0;
        void* arr[3] = {d->f, d->M, d->fresh};
        const size_t sizes[3] = {fb * 19 * ld, eb * 8 * ld, sizeof(int32_t)};
        for (int a = 0; a < 3; ++a) {
            if (hipMemcpyAsync(arr[a], (char*)snaps[k].buf + off, sizes[a],
                               hipMemcpyDeviceToDevice, p->stream) != hipSuccess &&
                st == LBM_OK)
                st = fail(LBM_ERR_DEVICE, "restore copy failed");
            off += sizes[a];
        }
        d->step = dstep0[k];
    }
    p->step = step0;
    if (hipStreamSynchronize(p->stream) != hipSuccess && st == LBM_OK)
        st = fail(LBM_ERR_DEVICE, "synchronise failed");
    for (const Snap& sn : snaps) p->dfree(sn.buf);
    p->grid = st == LBM_OK ? best : keep;
    p->order = st == LBM_OK ? best_order : keep_order;
    p->group_bytes = st == LBM_OK ? best_group : keep_group;
    p->drop_graph();
    p->dirty = true;                  // regroup at the next step
    if (st == LBM_OK && grid) *grid = p->grid;
    return st;
}

lbm_status lbm_pool_destroy(lbm_pool* p) {
    if (!p) return LBM_OK;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    for (int32_t s = 0; s < (int32_t)p->slots.size(); ++s)
        if (p->slots[s]) (void)lbm_pool_retire(p, s, nullptr);
    p->drop_graph();
    void* bufs[] = {p->d_doms, p->d_tile_first, p->d_tile_dom, p->d_ntiles, p->d_partials,
                    p->d_red, p->d_group_first, p->d_group_ntiles};
    for (void* b : bufs) p->dfree(b);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
    return LBM_OK;
}

}  // extern "C"
