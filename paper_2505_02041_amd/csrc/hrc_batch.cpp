// Batched forward + backward: many scenes of different power-of-two sizes in one
// HIP graph launch.  The scenes go to one persistent kernel that schedules
// their passes tile by tile; scenes from a size up (chosen by the autotuner,
// possibly none) instead run pass by pass as their own kernels in the same
// graph, where one pass fills the GPU and the persistent kernel's per-pass
// synchronisation costs more than the launch gaps it saves.  Tile sizes,
// kernel variant, claim chunk and that size are picked by timing candidates on
// the device.
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "../../include/hrc.h"
#include "hrc_internal.h"

using namespace hrc;

struct hrc_batch {
    int device = 0;
    char *dmem = nullptr;          // scene workspaces, then the scheduler tables
    size_t dmem_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int target_tiles = 0;          // chosen by the autotuner
    unsigned chunk = 1;            // items per claim, chosen by the autotuner
    int variant = 0;               // persistent kernel variant, chosen by the autotuner
    int grid = 0;
    int direct = 0;                // scenes run as their own kernels, chosen by the autotuner
};

namespace {

struct Plan {
    std::vector<Phase> phases;     // all scenes, each scene's passes in order
    std::vector<unsigned> seg_start;
    std::vector<int> seg_phase;
    std::vector<int> seg_step;
    std::vector<unsigned> step_items;
    unsigned total_items = 0;
};

// Elements per thread for a phase so that it splits into at most `target`
// tiles (tiles of 256*U outputs); fixed-shape phases keep their own tiles.
void size_tiles(Phase &p, int target) {
    if (p.kind == PH_SEED) p.a.seed.tile = 16;  // the persistent kernel's tiles
    if (p.kind == PH_TAIL) p.a.tail.tile = 16;
    if (p.kind == PH_SEED || p.kind == PH_SEED_ADJ || p.kind == PH_TAIL ||
        p.kind == PH_GATHER_ADJ)
        return;
    p.U = 1;
    unsigned t1 = phase_tiles(p);
    unsigned U = (t1 + (unsigned)target - 1) / (unsigned)target;
    p.U = (int)std::max(1u, std::min(U, 64u));
}

// The buffers a pass reads and writes (device base pointers: every level of a
// workspace and every field of a scene is its own buffer).  Pointers a pass
// carries but does not read at its level are left out.
void phase_access(const Phase &p, std::vector<const void *> &rd, std::vector<const void *> &wr) {
    rd.clear();
    wr.clear();
    auto r = [&](const void *q) { if (q) rd.push_back(q); };
    auto w = [&](const void *q) { if (q) wr.push_back(q); };
    switch (p.kind) {
        case PH_SEED: {
            const SeedArgs &a = p.a.seed;
            r(a.eps); r(a.sig);
            if (a.first <= 0) w(a.T0);
            if (a.first <= 1) w(a.T1);
            w(a.T2);
            break;
        }
        case PH_UP: r(p.a.up.Tp); w(p.a.up.T); break;
        case PH_DOWN: {
            const DownArgs &a = p.a.down;
            if (a.n + 1 < a.N) { r(a.Rn1); r(a.Tn1); }
            r(a.Tn);
            w(a.R);
            break;
        }
        case PH_TAIL: {
            const TailArgs &a = p.a.tail;
            r(a.eps); r(a.sig); r(a.R2);
            if (a.accumulate) r(a.out);
            w(a.out);
            break;
        }
        case PH_GATHER_ADJ: r(p.a.ga.dF); w(p.a.ga.dR0); break;
        case PH_DOWN_ADJ: {
            const DownAdjArgs &a = p.a.da;
            r(a.dR); r(a.Tn); r(a.Tn1);
            w(a.dRn1);
            break;
        }
        case PH_DT: {
            const DTArgs &a = p.a.dt;
            if (a.has_up) { r(a.Tn); r(a.dTn1); }
            if (a.n < a.N) { r(a.dRn); r(a.Rn); }
            if (a.n >= 1) r(a.dRm);
            if (a.n + 1 < a.N) r(a.Rn1);
            w(a.dT);
            break;
        }
        case PH_SEED_ADJ: {
            const SeedAdjArgs &a = p.a.sa;
            r(a.eps); r(a.sig); r(a.dT0); r(a.dT1); r(a.dT2);
            w(a.dE); w(a.dS);
            break;
        }
        case PH_BLUR:
        case PH_BLUR_ADJ: r(p.a.bl.in); r(p.a.bl.sig); w(p.a.bl.out); break;
        default: break;
    }
}

// Step of each pass of one scene's chain: one past the latest earlier pass it
// depends on (it reads what that pass wrote, or writes what that pass read or
// wrote), so independent passes (the reverse's merge-down adjoint beside the
// recomputed merge up and merge down) share a step.
std::vector<int> chain_steps(const std::vector<Phase> &chain) {
    std::vector<int> step(chain.size(), 0);
    std::vector<std::pair<const void *, int>> last_w, last_r;  // buffer, latest step
    auto find = [](std::vector<std::pair<const void *, int>> &v, const void *q) -> int * {
        for (auto &e : v)
            if (e.first == q) return &e.second;
        return nullptr;
    };
    std::vector<const void *> rd, wr;
    for (size_t i = 0; i < chain.size(); ++i) {
        phase_access(chain[i], rd, wr);
        int s = 0;
        for (const void *q : rd)
            if (int *t = find(last_w, q)) s = std::max(s, *t + 1);
        for (const void *q : wr) {
            if (int *t = find(last_w, q)) s = std::max(s, *t + 1);
            if (int *t = find(last_r, q)) s = std::max(s, *t + 1);
        }
        step[i] = s;
        for (const void *q : rd) {
            if (int *t = find(last_r, q)) *t = std::max(*t, s);
            else last_r.push_back({q, s});
        }
        for (const void *q : wr) {
            if (int *t = find(last_w, q)) *t = std::max(*t, s);
            else last_w.push_back({q, s});
        }
    }
    return step;
}

// Items in step order: step t holds, for every scene, its passes of step t
// (chain_steps), so every pass depends only on passes of earlier steps.
void order_items(Plan &pl, const std::vector<int> &first, const std::vector<int> &count,
                 const std::vector<std::vector<int>> &steps) {
    pl.seg_start.clear();
    pl.seg_phase.clear();
    pl.seg_step.clear();
    pl.step_items.clear();
    unsigned pos = 0;
    int max_step = -1;
    for (const auto &st : steps)
        for (int t : st) max_step = std::max(max_step, t);
    for (int t = 0; t <= max_step; ++t) {
        unsigned in_step = 0;
        for (size_t s = 0; s < first.size(); ++s) {
            for (int j = 0; j < count[s]; ++j) {
                if (steps[s][j] != t) continue;
                const int gi = first[s] + j;
                // whole groups of tiles; the bodies store nothing for tiles
                // past the phase's own count
                const unsigned tiles =
                    (phase_tiles(pl.phases[gi]) + kBatchQuarters - 1) / kBatchQuarters;
                pl.seg_start.push_back(pos);
                pl.seg_phase.push_back(gi);
                pl.seg_step.push_back(t);
                pos += tiles;
                in_step += tiles;
            }
        }
        pl.step_items.push_back(in_step);
    }
    pl.total_items = pos;
}

void free_batch(hrc_batch *b) {
    if (!b) return;
    DeviceGuard g(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dmem) (void)hipFree(b->dmem);
    delete b;
}

}  // namespace

extern "C" {

hrc_status hrc_batch_plan(hrc_context *ctx, const hrc_scene *scenes, int count, unsigned flags,
                          void *stream, hrc_batch **out) {
    if (!out) return HRC_ERR_INVALID_ARG;
    *out = nullptr;
    if (!scenes || count <= 0) return HRC_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i) {
        const hrc_scene &sc = scenes[i];
        if (sc.log2_size < HRC_MIN_LOG2 || sc.log2_size > HRC_MAX_LOG2) return HRC_ERR_SHAPE;
    }
    auto ok16 = [](const void *p) { return p && (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    for (int i = 0; i < count; ++i) {
        const hrc_scene &sc = scenes[i];
        if (!ok16(sc.emission) || !ok16(sc.sigma_t) || !ok16(sc.fluence)) return HRC_ERR_INVALID_ARG;
        const bool any = sc.grad_fluence || sc.grad_emission || sc.grad_sigma_t;
        if (any && (!ok16(sc.grad_fluence) || !ok16(sc.grad_emission) || !ok16(sc.grad_sigma_t)))
            return HRC_ERR_INVALID_ARG;
    }
    if ((flags & ~(HRC_FLAG_BATCH_FULL | HRC_FLAG_BATCH_DENSE | HRC_FLAG_BATCH_PERSISTENT)) ||
        (flags & (HRC_FLAG_BATCH_FULL | HRC_FLAG_BATCH_DENSE)) ==
            (HRC_FLAG_BATCH_FULL | HRC_FLAG_BATCH_DENSE))
        return HRC_ERR_UNSUPPORTED;
    if (!ctx) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    hipStream_t user = static_cast<hipStream_t>(stream);
    // the autotuner runs the batch on the caller's buffers: let pending work on
    // them finish first
    if (hipStreamSynchronize(user) != hipSuccess) return HRC_ERR_HIP;

    hrc_batch *b = new hrc_batch();
    b->device = ctx->device;

    // ---- device memory: per-scene workspaces, then scheduler tables --------
    std::vector<Layout> layouts(count);
    std::vector<size_t> ws_off(count);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const bool bwd = scenes[i].grad_fluence != nullptr;
        layouts[i] = make_layout(scenes[i].log2_size, bwd);
        ws_off[i] = off;
        off += align256(layouts[i].total);
    }
    const size_t ws_total = off;
    const size_t max_phases = (size_t)count * kMaxPhases;
    const size_t phases_off = ws_total;
    off += align256(max_phases * sizeof(Phase));
    const size_t seg_start_off = off;
    off += align256(max_phases * sizeof(unsigned));
    const size_t seg_phase_off = off;
    off += align256(max_phases * sizeof(int));
    const size_t seg_step_off = off;
    off += align256(max_phases * sizeof(int));
    const size_t step_items_off = off;
    off += align256(kMaxPhases * sizeof(unsigned));
    const size_t sched_off = off;  // claim counter, error word, one count per step
    off += align256(sched_words(kMaxPhases) * sizeof(unsigned));
    b->dmem_bytes = off;
    if (hipMalloc(&b->dmem, b->dmem_bytes) != hipSuccess) {
        b->dmem = nullptr;
        free_batch(b);
        return HRC_ERR_HIP;
    }

    // ---- phase chains: each scene's passes (the persistent kernel's copies get
    // its own tile sizes; the direct ones keep the standalone kernels')
    std::vector<std::vector<Phase>> chains(count);
    for (int i = 0; i < count; ++i) {
        const hrc_scene &sc = scenes[i];
        Ws w{b->dmem + ws_off[i], layouts[i]};
        SolveBuffers sb{sc.emission, sc.sigma_t, sc.fluence, sc.grad_fluence, sc.grad_emission,
                        sc.grad_sigma_t};
        Phase tmp[kMaxPhases];
        const int n = build_solve_phases(w, sb, sc.grad_fluence != nullptr, nullptr, tmp,
                                         kMaxPhases);
        chains[i].assign(tmp, tmp + n);
    }
    std::vector<std::vector<int>> steps(count);
    for (int i = 0; i < count; ++i) steps[i] = chain_steps(chains[i]);
    // scenes of log2 size >= min_direct run as their own kernels
    Plan pl;
    std::vector<int> first, np;
    std::vector<std::vector<int>> psteps;  // steps of the persistent kernel's scenes
    std::vector<const Phase *> direct_list;
    int n_direct = 0;
    auto split = [&](int min_direct) {
        pl = Plan();
        first.clear();
        np.clear();
        psteps.clear();
        direct_list.clear();
        n_direct = 0;
        for (int i = 0; i < count; ++i) {
            if (scenes[i].log2_size >= min_direct) {
                ++n_direct;
                for (const Phase &p : chains[i]) direct_list.push_back(&p);
            } else {
                first.push_back((int)pl.phases.size());
                np.push_back((int)chains[i].size());
                psteps.push_back(steps[i]);
                pl.phases.insert(pl.phases.end(), chains[i].begin(), chains[i].end());
            }
        }
    };

    int grids[kPersistentVariants];  // resident blocks of each kernel variant
    for (int v = 0; v < kPersistentVariants; ++v) {
        int per_cu = 0;
        if (persistent_occupancy(v, &per_cu) != hipSuccess || per_cu <= 0) per_cu = 1;
        grids[v] = ctx->num_cus * per_cu;
    }

    Phase *d_phases = reinterpret_cast<Phase *>(b->dmem + phases_off);
    unsigned *d_seg_start = reinterpret_cast<unsigned *>(b->dmem + seg_start_off);
    int *d_seg_phase = reinterpret_cast<int *>(b->dmem + seg_phase_off);
    int *d_seg_step = reinterpret_cast<int *>(b->dmem + seg_step_off);
    unsigned *d_step_items = reinterpret_cast<unsigned *>(b->dmem + step_items_off);
    unsigned *d_sched = reinterpret_cast<unsigned *>(b->dmem + sched_off);

    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        free_batch(b);
        return HRC_ERR_HIP;
    }
    BatchTables tables{};
    auto upload = [&](int target, unsigned chunk) -> bool {
        if (pl.phases.empty()) return true;
        for (Phase &p : pl.phases) size_tiles(p, target);
        order_items(pl, first, np, psteps);
        tables = BatchTables{d_phases, d_seg_start, d_seg_phase, d_seg_step, d_step_items,
                             (int)pl.seg_start.size(), (int)pl.step_items.size(), pl.total_items,
                             chunk};
        auto h2d = [&](void *dst, const void *src, size_t bytes) {
            return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, cap) == hipSuccess;
        };
        return h2d(d_phases, pl.phases.data(), pl.phases.size() * sizeof(Phase)) &&
               h2d(d_seg_start, pl.seg_start.data(), pl.seg_start.size() * sizeof(unsigned)) &&
               h2d(d_seg_phase, pl.seg_phase.data(), pl.seg_phase.size() * sizeof(int)) &&
               h2d(d_seg_step, pl.seg_step.data(), pl.seg_step.size() * sizeof(int)) &&
               h2d(d_step_items, pl.step_items.data(), pl.step_items.size() * sizeof(unsigned)) &&
               hipStreamSynchronize(cap) == hipSuccess;
    };
    int variant = 0;
    // one batch: the direct scenes' passes in order, then the persistent kernel
    auto run = [&]() -> bool {
        for (const Phase *p : direct_list)
            if (launch_phase(*p, cap) != hipSuccess) return false;
        if (pl.phases.empty()) return true;
        return launch_persistent(tables, d_sched, grids[variant], variant, cap) == hipSuccess;
    };

    // ---- autotune: which sizes run as their own kernels, the persistent
    // kernel variant (registers vs resident blocks), the tile count per phase
    // (hence elements per tile) as a multiple of the resident tile slots, and
    // the claim chunk: the fastest whole-batch launch wins -------------------
    std::vector<int> min_directs{HRC_MAX_LOG2 + 1};  // none direct
    if (!(flags & HRC_FLAG_BATCH_PERSISTENT)) {
        // from 256^2 up: below, a pass does not fill the GPU
        for (int L = HRC_MAX_LOG2; L >= 8; --L)
            for (int i = 0; i < count; ++i)
                if (scenes[i].log2_size == L) {
                    min_directs.push_back(L);
                    break;
                }
    }
    const int mults[] = {1, 2, 4};
    const unsigned chunks[] = {1u, 4u};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool fine = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    float best_ms = 1e30f;
    int best = grids[0] * kBatchQuarters, best_variant = 0, best_min = HRC_MAX_LOG2 + 1;
    unsigned best_chunk = 1;
    auto time_one = [&](int min_direct, int v, int target, unsigned ch) {
        fine = upload(target, ch) && run() && hipStreamSynchronize(cap) == hipSuccess;  // warm-up
        if (!fine) return;
        fine = hipEventRecord(e0, cap) == hipSuccess && run() &&
               hipEventRecord(e1, cap) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (fine && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = target;
            best_chunk = ch;
            best_variant = v;
            best_min = min_direct;
        }
    };
    for (int min_direct : min_directs) {
        if (!fine) break;
        split(min_direct);
        if (pl.phases.empty()) {  // every scene direct: nothing to tune
            const int v = (flags & HRC_FLAG_BATCH_DENSE) ? 1 : 0;
            time_one(min_direct, v, grids[v] * kBatchQuarters, 1u);
            continue;
        }
        for (int v = 0; v < kPersistentVariants && fine; ++v) {
            if ((flags & HRC_FLAG_BATCH_FULL) && v != 0) continue;
            if ((flags & HRC_FLAG_BATCH_DENSE) && v != 1) continue;
            variant = v;
            for (int mult : mults)
                for (unsigned ch : chunks)
                    if (fine) time_one(min_direct, v, grids[v] * kBatchQuarters * mult, ch);
        }
        if (fine) {
            // the scheduler's error word (a dependency wait that timed out)
            unsigned err = 0;
            fine = hipMemcpy(&err, d_sched + kSchedStride, sizeof(unsigned),
                             hipMemcpyDeviceToHost) == hipSuccess && err == 0;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    split(best_min);
    b->direct = n_direct;
    b->target_tiles = best;
    b->chunk = best_chunk;
    b->variant = variant = best_variant;
    b->grid = grids[variant];
    if (fine) fine = upload(best, best_chunk);

    // ---- capture one launch in a graph ---------------------------------
    if (fine) fine = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (fine) {
        bool launched = run();
        fine = (hipStreamEndCapture(cap, &b->graph) == hipSuccess) && launched;
    }
    if (fine) fine = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
    (void)hipStreamDestroy(cap);
    if (!fine) {
        free_batch(b);
        return HRC_ERR_HIP;
    }
    *out = b;
    return HRC_OK;
}

hrc_status hrc_batch_launch(hrc_batch *batch, void *stream) {
    if (!batch || !batch->exec) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(batch->device);
    if (!g.ok) return HRC_ERR_HIP;
    return hipGraphLaunch(batch->exec, static_cast<hipStream_t>(stream)) == hipSuccess
               ? HRC_OK
               : HRC_ERR_HIP;
}

size_t hrc_batch_workspace_bytes(const hrc_batch *batch) {
    return batch ? batch->dmem_bytes : 0;
}

hrc_status hrc_batch_describe(const hrc_batch *batch, int *variant, int *grid,
                              int *target_tiles, int *chunk, int *direct_scenes) {
    if (!batch) return HRC_ERR_INVALID_ARG;
    if (direct_scenes) *direct_scenes = batch->direct;
    if (variant) *variant = batch->variant;
    if (grid) *grid = batch->grid;
    if (target_tiles) *target_tiles = batch->target_tiles;
    if (chunk) *chunk = (int)batch->chunk;
    return HRC_OK;
}

void hrc_batch_destroy(hrc_batch *batch) { free_batch(batch); }

}  // extern "C"
