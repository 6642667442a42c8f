// Batched forward + backward: many scenes of different power-of-two sizes in one
// HIP graph launch.  The scenes go to one persistent kernel that schedules
// their passes tile by tile, one queue per XCD, each scene pinned to one
// queue; scenes from a size up (chosen by the autotuner, possibly none) can
// instead run pass by pass as their own kernels in the same graph, ahead of
// the persistent kernel.  The queues' scene lists, how many scenes of a queue
// share a workspace slot, the tile sizes, kernel variant and claim chunk are
// picked by timing candidates on the device.
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/hrc.h"
#include "hrc_internal.h"

using namespace hrc;

struct hrc_batch {
    int device = 0;
    char *dmem = nullptr;          // the scenes' workspaces
    size_t dmem_bytes = 0;
    char *tmem = nullptr;          // scheduler tables and words
    size_t tmem_bytes = 0;
    unsigned *sched = nullptr;     // scheduler words inside tmem
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int target_tiles = 0;          // chosen by the autotuner
    unsigned chunk = 1;            // items per claim, chosen by the autotuner
    int variant = 0;               // persistent kernel variant, chosen by the autotuner
    int grid = 0;
    int direct = 0;                // scenes run as their own kernels, chosen by the autotuner
    int queues = 0;                // queues of the persistent kernel
    int xcd_local = 0;             // one queue per XCD
    int slots = 0;                 // workspace slots per queue (0: one per scene)
    int branches = 1;              // graph branches the direct scenes run in
    std::vector<int> cand_desc;    // every timed candidate: kCandFields ints each
    std::vector<float> cand_ms;    // and its time
};

// Fields of a timed candidate as hrc_batch_candidates reports them.
constexpr int kCandFields = 8;

namespace {

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

// One arrangement of the batch: which scenes run as their own kernels, how the
// others are spread over queues and workspace slots, and the resulting tables.
struct Arrangement {
    int min_direct = HRC_MAX_LOG2 + 1;  // scenes of this log2 size and up run direct
    int nqueues = 1;
    int slots = 0;                      // workspace slots per queue; 0 = one per scene
    int target = 0;                     // tiles per phase
    int quarters = kMaxQuarters;        // tiles per group (per block of the kernel variant)
    int branches = 1;                   // graph branches the direct scenes run in
    std::vector<Phase> direct[kMaxBranches];  // each branch's direct passes, in order
    std::vector<Phase> phases;          // the persistent kernel's passes
    std::vector<unsigned> seg_start;
    std::vector<int> seg_phase, seg_step;
    std::vector<unsigned> step_items;
    int q_seg[kMaxQueues + 1] = {};
    int q_step[kMaxQueues + 1] = {};
    unsigned q_items[kMaxQueues] = {};
    int n_direct = 0;
    size_t ws_bytes = 0;                // workspace the arrangement needs
    std::vector<int> phase_scene;       // scene of each persistent pass
    std::vector<int> scene_slot;        // workspace slot of each scene (-1: direct)
    std::vector<size_t> slot_base;      // byte offset of each slot in the workspace
};

// Relative amount of work of a scene: its pixels times its passes.
double scene_cost(const hrc_scene &sc) {
    const double S = double(1 << sc.log2_size);
    return S * S * (sc.grad_fluence ? 2.0 : 1.0) * (sc.log2_size + 2);
}

// Lays out the workspaces at `base` and builds the tables of an arrangement
// (with a null base: only the workspace size, ws_bytes).
// The direct scenes run one after another, so they share one workspace; the
// persistent kernel runs after them, so its slots reuse the same memory.  A
// queue's scenes (largest first, greedily balanced over the queues by cost)
// go round-robin to its slots; the scenes of one slot run one after another
// (a scene's first step follows the previous one's last), scenes of different
// slots side by side, and within a scene independent passes share a step.
// Step t of a queue holds, for every scene of the queue in order, its passes
// of step t.
void arrange(Arrangement &ar, const hrc_scene *scenes, int count, char *base) {
    for (auto &d : ar.direct) d.clear();
    ar.phases.clear();
    ar.phase_scene.clear();
    ar.seg_start.clear();
    ar.seg_phase.clear();
    ar.seg_step.clear();
    ar.step_items.clear();
    ar.n_direct = 0;
    std::vector<Layout> lay(count);
    for (int i = 0; i < count; ++i)
        lay[i] = make_layout(scenes[i].log2_size, scenes[i].grad_fluence != nullptr);
    auto solve = [&](int i, char *ws, bool persistent, std::vector<Phase> &out) {
        const hrc_scene &sc = scenes[i];
        SolveBuffers sb{sc.emission, sc.sigma_t, sc.fluence, sc.grad_fluence, sc.grad_emission,
                        sc.grad_sigma_t};
        Phase tmp[kMaxPhases];
        const int n = build_solve_phases(Ws{ws, lay[i]}, sb, sc.grad_fluence != nullptr, nullptr,
                                         tmp, kMaxPhases);
        out.assign(tmp, tmp + n);
        if (persistent)
            for (Phase &p : out) size_tiles(p, ar.target);
    };
    // direct scenes, in the caller's order, in one shared workspace per branch
    // (with two branches: largest first, each to the lighter branch)
    std::vector<int> pers, direct;
    for (int i = 0; i < count; ++i) {
        if (scenes[i].log2_size >= ar.min_direct) direct.push_back(i);
        else pers.push_back(i);
    }
    ar.n_direct = (int)direct.size();
    const int nbr = std::max(1, std::min({ar.branches, kMaxBranches, (int)direct.size()}));
    std::vector<int> branch_of(count, 0);
    if (nbr > 1) {
        std::vector<int> order = direct;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return scene_cost(scenes[a]) > scene_cost(scenes[b]);
        });
        double load[kMaxBranches] = {};
        for (int i : order) {
            const int bb = (int)(std::min_element(load, load + nbr) - load);
            branch_of[i] = bb;
            load[bb] += scene_cost(scenes[i]);
        }
    }
    size_t branch_off[kMaxBranches + 1] = {};
    {
        size_t branch_bytes[kMaxBranches] = {};
        for (int i : direct)
            branch_bytes[branch_of[i]] = std::max(branch_bytes[branch_of[i]], align256(lay[i].total));
        for (int bb = 0; bb < kMaxBranches; ++bb) branch_off[bb + 1] = branch_off[bb] + branch_bytes[bb];
    }
    const size_t direct_bytes = branch_off[kMaxBranches];
    // persistent scenes: largest first, each to the least-loaded queue
    std::stable_sort(pers.begin(), pers.end(), [&](int a, int b) {
        return scene_cost(scenes[a]) > scene_cost(scenes[b]);
    });
    const int nq = ar.nqueues;
    std::vector<std::vector<int>> queue(nq);
    std::vector<double> load(nq, 0.0);
    for (int i : pers) {
        const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        queue[q].push_back(i);
        load[q] += scene_cost(scenes[i]);
    }
    // slots: sized to the largest scene they hold, laid out queue by queue
    size_t off = 0;
    std::vector<int> slot_of(count, -1);
    std::vector<size_t> slot_base;
    for (int q = 0; q < nq; ++q) {
        const int n = (int)queue[q].size();
        if (n == 0) continue;
        const int k = ar.slots > 0 ? std::min(ar.slots, n) : n;
        std::vector<size_t> size(k, 0);
        for (int j = 0; j < n; ++j)
            size[j % k] = std::max(size[j % k], align256(lay[queue[q][j]].total));
        for (int j = 0; j < n; ++j) slot_of[queue[q][j]] = (int)slot_base.size() + j % k;
        for (int s = 0; s < k; ++s) {
            slot_base.push_back(off);
            off += size[s];
        }
    }
    ar.ws_bytes = std::max(direct_bytes, off);
    ar.scene_slot = slot_of;
    ar.slot_base = slot_base;
    if (!base) return;  // sizes only
    std::vector<Phase> chain;
    for (int i : direct) {
        solve(i, base + branch_off[branch_of[i]], false, chain);
        ar.direct[branch_of[i]].insert(ar.direct[branch_of[i]].end(), chain.begin(), chain.end());
    }
    // per queue: each scene's steps, offset past the previous scene of its slot
    int total_steps = 0, seg = 0;
    for (int q = 0; q < nq; ++q) {
        ar.q_seg[q] = seg;
        ar.q_step[q] = total_steps;
        const int n = (int)queue[q].size();
        std::vector<std::vector<Phase>> chains(n);
        std::vector<std::vector<int>> steps(n);
        std::vector<int> first(n);
        std::vector<int> slot_next(slot_base.size(), 0);  // first free step of each slot
        int nsteps = 0;
        for (int j = 0; j < n; ++j) {
            const int i = queue[q][j];
            solve(i, base + slot_base[slot_of[i]], true, chains[j]);
            steps[j] = chain_steps(chains[j]);
            const int o = slot_next[slot_of[i]];
            int last = o;
            for (int &t : steps[j]) {
                t += o;
                last = std::max(last, t);
            }
            slot_next[slot_of[i]] = last + 1;
            nsteps = std::max(nsteps, last + 1);
            first[j] = (int)ar.phases.size();
            ar.phases.insert(ar.phases.end(), chains[j].begin(), chains[j].end());
            ar.phase_scene.insert(ar.phase_scene.end(), chains[j].size(), i);
        }
        unsigned pos = 0;
        for (int t = 0; t < nsteps; ++t) {
            unsigned in_step = 0;
            for (int j = 0; j < n; ++j) {
                for (size_t k = 0; k < chains[j].size(); ++k) {
                    if (steps[j][k] != t) continue;
                    const int gi = first[j] + (int)k;
                    // whole groups of tiles; the bodies store nothing for tiles
                    // past the phase's own count
                    const unsigned groups =
                        (phase_tiles(ar.phases[gi]) + ar.quarters - 1) / ar.quarters;
                    ar.seg_start.push_back(pos);
                    ar.seg_phase.push_back(gi);
                    ar.seg_step.push_back(t);
                    pos += groups;
                    in_step += groups;
                    ++seg;
                }
            }
            ar.step_items.push_back(in_step);
        }
        ar.q_items[q] = pos;
        total_steps += nsteps;
    }
    ar.q_seg[nq] = seg;
    ar.q_step[nq] = total_steps;
}

void free_batch(hrc_batch *b) {
    if (!b) return;
    DeviceGuard g(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->tmem) (void)hipFree(b->tmem);
    delete b;
}

// Queues the persistent kernel can use on this device with `grid` blocks: the
// number of XCDs if every XCD runs at least one block of the grid (probed),
// else 0.
int probe_xcds(int grid, int variant, unsigned *dbuf, hipStream_t s) {
    if (launch_xcd_probe(dbuf, grid, variant, s) != hipSuccess) return 0;
    std::vector<unsigned> h(grid);
    if (hipMemcpyAsync(h.data(), dbuf, grid * sizeof(unsigned), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return 0;
    unsigned hi = 0;
    for (unsigned x : h) hi = std::max(hi, x);
    if (hi >= (unsigned)kMaxQueues) return 0;
    std::vector<int> per(hi + 1, 0);
    for (unsigned x : h) ++per[x];
    for (int c : per)
        if (c == 0) return 0;
    return (int)hi + 1;
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

    // ---- device memory: scheduler tables (sized for the most phases and
    // steps any arrangement can have), then the workspace of the arrangement
    // that needs the most (every persistent scene in a slot of its own) ------
    const size_t max_phases = (size_t)count * kMaxPhases;
    size_t off = 0;
    const size_t phases_off = off;
    off += align256(max_phases * sizeof(Phase));
    const size_t seg_start_off = off;
    off += align256(max_phases * sizeof(unsigned));
    const size_t seg_phase_off = off;
    off += align256(max_phases * sizeof(int));
    const size_t seg_step_off = off;
    off += align256(max_phases * sizeof(int));
    const size_t step_items_off = off;
    off += align256(max_phases * sizeof(unsigned));
    const size_t sched_off = off;
    off += align256(sched_words(kMaxQueues, (int)max_phases) * sizeof(unsigned));
    constexpr int kMaxProbe = 1 << 14;  // blocks of a probed grid
    const size_t probe_off = off;
    off += align256(kMaxProbe * sizeof(unsigned));
    b->tmem_bytes = off;
    size_t ws_max = 0;
    for (int i = 0; i < count; ++i)
        ws_max += align256(make_layout(scenes[i].log2_size, scenes[i].grad_fluence != nullptr).total);
    if (hipMalloc(&b->tmem, b->tmem_bytes) != hipSuccess) {
        b->tmem = nullptr;
        free_batch(b);
        return HRC_ERR_HIP;
    }
    if (hipMalloc(&b->dmem, ws_max) != hipSuccess) {
        b->dmem = nullptr;
        free_batch(b);
        return HRC_ERR_HIP;
    }
    b->dmem_bytes = ws_max;
    Phase *d_phases = reinterpret_cast<Phase *>(b->tmem + phases_off);
    unsigned *d_seg_start = reinterpret_cast<unsigned *>(b->tmem + seg_start_off);
    int *d_seg_phase = reinterpret_cast<int *>(b->tmem + seg_phase_off);
    int *d_seg_step = reinterpret_cast<int *>(b->tmem + seg_step_off);
    unsigned *d_step_items = reinterpret_cast<unsigned *>(b->tmem + step_items_off);
    b->sched = reinterpret_cast<unsigned *>(b->tmem + sched_off);
    // error word and wait configuration start at zero (outside any graph)
    if (hipMemset(b->sched, 0, (size_t)kSchedExit * kSchedStride * sizeof(unsigned)) !=
        hipSuccess) {
        free_batch(b);
        return HRC_ERR_HIP;
    }

    // the capture stream, one more stream per extra graph branch, and the
    // events that fork the branches from it and join them again
    hipStream_t cap = nullptr, side[kMaxBranches] = {};
    hipEvent_t fork = nullptr, join[kMaxBranches] = {};
    auto free_streams = [&]() {
        if (cap) (void)hipStreamDestroy(cap);
        if (fork) (void)hipEventDestroy(fork);
        for (int i = 1; i < kMaxBranches; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
        }
    };
    bool streams_ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess &&
                      hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 1; streams_ok && i < kMaxBranches; ++i)
        streams_ok = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking) == hipSuccess &&
                     hipEventCreateWithFlags(&join[i], hipEventDisableTiming) == hipSuccess;
    if (!streams_ok) {
        free_streams();
        free_batch(b);
        return HRC_ERR_HIP;
    }

    // resident blocks of each kernel variant, and the XCDs their grids reach
    int grids[kPersistentVariants], xcds[kPersistentVariants];
    for (int v = 0; v < kPersistentVariants; ++v) {
        int per_cu = 0;
        if (persistent_occupancy(v, &per_cu) != hipSuccess || per_cu <= 0) per_cu = 1;
        grids[v] = ctx->num_cus * per_cu;
        xcds[v] = grids[v] <= kMaxProbe
                      ? probe_xcds(grids[v], v, reinterpret_cast<unsigned *>(b->tmem + probe_off),
                                   cap)
                      : 0;
    }

    Arrangement ar;
    BatchTables tables{};
    int variant = 0;
    unsigned chunk = 1;
    bool xcd_local = false;
    auto upload = [&]() -> bool {
        tables = BatchTables{};
        tables.phases = d_phases;
        tables.seg_start = d_seg_start;
        tables.seg_phase = d_seg_phase;
        tables.seg_step = d_seg_step;
        tables.step_items = d_step_items;
        tables.nqueues = ar.nqueues;
        tables.xcd_local = xcd_local ? 1 : 0;
        for (int q = 0; q <= ar.nqueues; ++q) {
            tables.q_seg[q] = ar.q_seg[q];
            tables.q_step[q] = ar.q_step[q];
        }
        for (int q = 0; q < ar.nqueues; ++q) tables.q_items[q] = ar.q_items[q];
        tables.chunk = chunk;
        if (ar.phases.empty()) return true;
        auto h2d = [&](void *dst, const void *src, size_t bytes) {
            return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, cap) == hipSuccess;
        };
        return h2d(d_phases, ar.phases.data(), ar.phases.size() * sizeof(Phase)) &&
               h2d(d_seg_start, ar.seg_start.data(), ar.seg_start.size() * sizeof(unsigned)) &&
               h2d(d_seg_phase, ar.seg_phase.data(), ar.seg_phase.size() * sizeof(int)) &&
               h2d(d_seg_step, ar.seg_step.data(), ar.seg_step.size() * sizeof(int)) &&
               h2d(d_step_items, ar.step_items.data(), ar.step_items.size() * sizeof(unsigned)) &&
               hipStreamSynchronize(cap) == hipSuccess;
    };
    // one batch: the direct scenes' passes in order, then the persistent kernel
    auto run = [&]() -> bool {
        // branches 1.. fork from the stream and join it again before the
        // persistent kernel; branch 0 runs on the stream itself
        bool forked = false;
        for (int i = 1; i < kMaxBranches; ++i) {
            if (ar.direct[i].empty()) continue;
            if (!forked && hipEventRecord(fork, cap) != hipSuccess) return false;
            forked = true;
            if (hipStreamWaitEvent(side[i], fork, 0) != hipSuccess) return false;
            for (const Phase &p : ar.direct[i])
                if (launch_phase(p, side[i]) != hipSuccess) return false;
        }
        for (const Phase &p : ar.direct[0])
            if (launch_phase(p, cap) != hipSuccess) return false;
        for (int i = 1; i < kMaxBranches; ++i) {
            if (ar.direct[i].empty()) continue;
            if (hipEventRecord(join[i], side[i]) != hipSuccess ||
                hipStreamWaitEvent(cap, join[i], 0) != hipSuccess)
                return false;
        }
        if (ar.phases.empty()) return true;
        return launch_persistent(tables, b->sched, grids[variant], variant, cap) == hipSuccess;
    };

    // ---- autotune.  A candidate is a split (which sizes run direct), a queue
    // layout (one queue per XCD, or one queue over the whole device), the
    // workspace slots per queue, the kernel variant, the tile count per phase
    // (a multiple of the resident tile slots per queue) and the claim chunk.
    // Stage 1 times every split, queue layout, slot count and variant at one
    // setting of the rest; stage 2 sweeps the rest for the winner.  The fastest
    // whole-batch launch wins. ------------------------------------------------
    struct Cand {
        int min_direct, xcd, slots, variant, mult;
        unsigned chunk;
        int branches = 1;
    };
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
    std::vector<int> variants;
    for (int v = 0; v < kPersistentVariants; ++v) {
        // variants 0, 2: full register budget; 1, 3: 64 VGPRs
        if ((flags & HRC_FLAG_BATCH_FULL) && v % 2 != 0) continue;
        if ((flags & HRC_FLAG_BATCH_DENSE) && v % 2 != 1) continue;
        variants.push_back(v);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool fine = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    bool timed_out = false;
    float best_ms = 1e30f;
    Cand best{HRC_MAX_LOG2 + 1, 0, 0, variants[0], 1, 1u};
    auto set_up = [&](const Cand &c) -> bool {
        variant = c.variant;
        chunk = c.chunk;
        xcd_local = c.xcd > 0;
        ar = Arrangement();
        ar.min_direct = c.min_direct;
        ar.branches = c.branches;
        ar.nqueues = xcd_local ? c.xcd : 1;
        ar.slots = c.slots;
        ar.quarters = persistent_quarters(variant);
        ar.target = std::max(1, grids[variant] / ar.nqueues) * ar.quarters * c.mult;
        arrange(ar, scenes, count, b->dmem);
        return ar.ws_bytes <= b->dmem_bytes && upload();
    };
    auto time_one = [&](const Cand &c) {
        if (!fine) return;
        fine = set_up(c) && run() && hipStreamSynchronize(cap) == hipSuccess;  // warm-up
        if (!fine) return;
        fine = hipEventRecord(e0, cap) == hipSuccess && run() &&
               hipEventRecord(e1, cap) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (!fine || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            fine = false;
            return;
        }
        // the scheduler's error word (a dependency wait that gave up)
        unsigned err = 0;
        fine = hipMemcpy(&err, b->sched + kSchedError * kSchedStride, sizeof(unsigned),
                         hipMemcpyDeviceToHost) == hipSuccess;
        if (fine && err) {
            timed_out = true;
            fine = false;
            return;
        }
        const int desc[kCandFields] = {c.min_direct <= HRC_MAX_LOG2 ? c.min_direct : 0,
                                       ar.nqueues, xcd_local ? 1 : 0, c.slots, c.variant,
                                       ar.target, (int)c.chunk, c.branches};
        b->cand_desc.insert(b->cand_desc.end(), desc, desc + kCandFields);
        b->cand_ms.push_back(ms);
        // more graph branches (a workspace more each) must win by 1%
        if (c.branches > best.branches ? ms < 0.99f * best_ms : ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    };
    // per-XCD queues when every variant's grid reaches the same XCDs
    int xcd_q = xcds[0];
    for (int v = 1; v < kPersistentVariants; ++v)
        if (xcds[v] != xcd_q) xcd_q = 0;
    const int xcd_opts[] = {xcd_q > 1 ? xcd_q : 0, 0};
    for (int md : min_directs) {
        bool all_direct = true;
        for (int i = 0; i < count; ++i) all_direct = all_direct && scenes[i].log2_size >= md;
        if (all_direct) {  // nothing for the persistent kernel: one timing
            time_one(Cand{md, 0, 0, variants[0], 2, 1u});
            continue;
        }
        for (int xo = 0; xo < 2; ++xo) {
            if (xo == 1 && xcd_opts[0] == 0) continue;  // the single queue is tried once
            const int xc = xcd_opts[xo];
            for (int slots : {1, 2, 0})
                for (int v : variants) time_one(Cand{md, xc, slots, v, 2, 1u});
        }
    }
    const Cand stage1 = best;
    bool stage1_direct = true;
    for (int i = 0; i < count; ++i)
        stage1_direct = stage1_direct && scenes[i].log2_size >= stage1.min_direct;
    if (!stage1_direct)
        for (int mult : {1, 2, 4})
            for (unsigned ch : {1u, 4u})
                if (!(mult == stage1.mult && ch == stage1.chunk))
                    time_one(Cand{stage1.min_direct, stage1.xcd, stage1.slots, stage1.variant, mult,
                                  ch});
    // stage 3: the direct scenes in 2 or 4 graph branches (each with a
    // workspace of its own), so that one branch's passes fill the GPU where
    // another's drain and ramp at a kernel boundary
    {
        int n_direct = 0;
        for (int i = 0; i < count; ++i) n_direct += scenes[i].log2_size >= best.min_direct ? 1 : 0;
        const Cand stage2 = best;
        for (int br : {2, 4})
            if (br <= n_direct) {
                Cand c = stage2;
                c.branches = br;
                time_one(c);
            }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);

    // ---- the winner: its own (smaller) workspace, tables, and the graph ----
    if (fine) {
        ar = Arrangement();
        ar.min_direct = best.min_direct;
        ar.branches = best.branches;
        ar.nqueues = best.xcd > 0 ? best.xcd : 1;
        ar.slots = best.slots;
        ar.quarters = persistent_quarters(best.variant);
        ar.target = std::max(1, grids[best.variant] / ar.nqueues) * ar.quarters * best.mult;
        arrange(ar, scenes, count, nullptr);  // sizes only
        if (ar.ws_bytes < b->dmem_bytes) {
            (void)hipFree(b->dmem);
            b->dmem = nullptr;
            b->dmem_bytes = 0;
            if (hipMalloc(&b->dmem, std::max<size_t>(ar.ws_bytes, 256)) != hipSuccess) {
                b->dmem = nullptr;
                fine = false;
            } else {
                b->dmem_bytes = std::max<size_t>(ar.ws_bytes, 256);
            }
        }
    }
    if (fine) fine = set_up(best);
    b->direct = ar.n_direct;
    b->target_tiles = ar.target;
    b->chunk = best.chunk;
    b->variant = best.variant;
    b->grid = grids[best.variant];
    b->queues = ar.nqueues;
    b->xcd_local = best.xcd > 0 ? 1 : 0;
    b->slots = best.slots;
    b->branches = ar.direct[1].empty() ? 1 : best.branches;

    // ---- capture one launch in a graph ---------------------------------
    if (fine) fine = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (fine) {
        bool launched = run();
        fine = (hipStreamEndCapture(cap, &b->graph) == hipSuccess) && launched;
    }
    if (fine) fine = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
    free_streams();
    if (!fine) {
        free_batch(b);
        return timed_out ? HRC_ERR_TIMEOUT : HRC_ERR_HIP;
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

hrc_status hrc_batch_status(hrc_batch *batch, void *stream) {
    if (!batch || !batch->sched) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(batch->device);
    if (!g.ok) return HRC_ERR_HIP;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return HRC_ERR_HIP;
    unsigned err = 0;
    unsigned *word = batch->sched + kSchedError * kSchedStride;
    if (hipMemcpy(&err, word, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
        return HRC_ERR_HIP;
    if (!err) return HRC_OK;
    const unsigned zero = 0;
    if (hipMemcpy(word, &zero, sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess)
        return HRC_ERR_HIP;
    return HRC_ERR_TIMEOUT;
}

hrc_status hrc_batch_debug_waits(hrc_batch *batch, unsigned spins) {
    if (!batch || !batch->sched) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(batch->device);
    if (!g.ok) return HRC_ERR_HIP;
    const unsigned cfg[2] = {spins, spins ? 1u : 0u};
    return hipMemcpy(batch->sched + kSchedConfig * kSchedStride, cfg, sizeof(cfg),
                     hipMemcpyHostToDevice) == hipSuccess
               ? HRC_OK
               : HRC_ERR_HIP;
}

size_t hrc_batch_workspace_bytes(const hrc_batch *batch) {
    return batch ? batch->dmem_bytes + batch->tmem_bytes : 0;
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

hrc_status hrc_batch_queues(const hrc_batch *batch, int *queues, int *xcd_local, int *slots,
                            int *branches) {
    if (!batch) return HRC_ERR_INVALID_ARG;
    if (queues) *queues = batch->queues;
    if (xcd_local) *xcd_local = batch->xcd_local;
    if (slots) *slots = batch->slots;
    if (branches) *branches = batch->branches;
    return HRC_OK;
}

hrc_status hrc_batch_candidates(const hrc_batch *batch, int max, int *count, int *desc,
                                float *ms) {
    if (!batch || !count || max < 0 || (max > 0 && (!desc || !ms))) return HRC_ERR_INVALID_ARG;
    const int n = (int)batch->cand_ms.size();
    *count = n;
    for (int i = 0; i < n && i < max; ++i) {
        for (int f = 0; f < kCandFields; ++f) desc[i * kCandFields + f] = batch->cand_desc[i * kCandFields + f];
        ms[i] = batch->cand_ms[i];
    }
    return HRC_OK;
}

void hrc_batch_destroy(hrc_batch *batch) { free_batch(batch); }

}  // extern "C"
