// Sanitizer driver for the library's host logic (test infrastructure).
// Compiled with AddressSanitizer and UndefinedBehaviorSanitizer on the host
// side, together with the library's sources (this file includes the batch
// planner's translation unit to reach its internal functions), it runs without
// a GPU: the C ABI's argument checks and workspace layouts, and the batch
// planner's arrangement of many scenes over queues and workspace slots on fake
// device addresses that are never dereferenced, checking that no two passes
// that touch the same buffer share a step and that each scene's dependencies
// keep their order.
#include "../../paper_2505_02041_amd/csrc/hrc_batch.cpp"

#include <cstdio>
#include <cstring>

static int fails = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

// Distinct fake device addresses, 256-byte aligned, 4 GiB apart.
static char *fake(size_t i) {
    return reinterpret_cast<char *>(static_cast<uintptr_t>((i + 1) << 32));
}

// The regions of a layout lie inside it, 256-byte aligned, and do not overlap.
static void check_layout(const Layout &L, bool backward, int iv = 8) {
    std::vector<std::pair<size_t, size_t>> reg;
    const size_t SS = L.S * L.S;
    for (int n = backward ? 0 : kTracedLevels - 1; n < L.N; ++n)
        reg.push_back({L.t_level[n], L.group * t_level_entries(L.N, n) * iv});
    for (int i = 0; i < L.r_count; ++i) reg.push_back({L.r_level[i], L.group * SS * 4});
    if (!backward) reg.push_back({L.aux, SS * 4});
    if (backward) {
        for (int n = 0; n <= L.N; ++n) reg.push_back({L.dt_level[n], 4 * t_level_entries(L.N, n) * 8});
        for (int i = 0; i < L.N; ++i) reg.push_back({L.dr_level[i], 4 * SS * 4});
    }
    std::sort(reg.begin(), reg.end());
    size_t end = 256;  // the validation flag
    for (auto &r : reg) {
        CHECK(r.first % 256 == 0);
        CHECK(r.first >= end);
        end = r.first + r.second;
    }
    CHECK(end <= L.total);
}

struct Access {
    std::vector<const void *> rd, wr;
};

static bool conflict(const Access &a, const Access &b) {
    auto has = [](const std::vector<const void *> &v, const void *p) {
        return std::find(v.begin(), v.end(), p) != v.end();
    };
    for (const void *p : a.wr)
        if (has(b.rd, p) || has(b.wr, p)) return true;
    for (const void *p : b.wr)
        if (has(a.rd, p)) return true;
    return false;
}

static void check_arrangement(const Arrangement &ar, const std::vector<hrc_scene> &sc) {
    const int count = (int)sc.size();
    const size_t np = ar.phases.size();
    std::vector<Access> acc(np);
    for (size_t a = 0; a < np; ++a) phase_access(ar.phases[a], acc[a].rd, acc[a].wr);
    // every persistent pass in exactly one segment; steps per queue consistent
    std::vector<int> seen(np, 0), step_of(np, -1), queue_of(np, -1);
    for (int q = 0; q < ar.nqueues; ++q) {
        unsigned items = 0;
        std::vector<unsigned> per_step(ar.q_step[q + 1] - ar.q_step[q], 0);
        for (int g = ar.q_seg[q]; g < ar.q_seg[q + 1]; ++g) {
            const int pi = ar.seg_phase[g];
            CHECK(pi >= 0 && pi < (int)np);
            ++seen[pi];
            step_of[pi] = ar.seg_step[g];
            queue_of[pi] = q;
            if (g > ar.q_seg[q]) CHECK(ar.seg_step[g] >= ar.seg_step[g - 1]);
            CHECK(ar.seg_start[g] == items);
            const unsigned groups = (phase_tiles(ar.phases[pi]) + ar.quarters - 1) / ar.quarters;
            items += groups;
            CHECK(ar.seg_step[g] >= 0 && ar.seg_step[g] < (int)per_step.size());
            per_step[ar.seg_step[g]] += groups;
        }
        CHECK(items == ar.q_items[q]);
        for (size_t t = 0; t < per_step.size(); ++t)
            CHECK(ar.step_items[ar.q_step[q] + t] == per_step[t]);
    }
    for (int v : seen) CHECK(v == 1);
    // graph branches of the direct scenes run side by side: no buffer that one
    // branch writes is touched by another
    for (int x = 0; x < kMaxBranches; ++x)
        for (int y = x + 1; y < kMaxBranches; ++y)
            for (const Phase &p : ar.direct[x])
                for (const Phase &q : ar.direct[y]) {
                    Access a, b;
                    phase_access(p, a.rd, a.wr);
                    phase_access(q, b.rd, b.wr);
                    CHECK(!conflict(a, b));
                }
    int direct_passes = 0;
    for (int x = 0; x < kMaxBranches; ++x) direct_passes += (int)ar.direct[x].size();
    if (ar.n_direct > 0) CHECK(direct_passes > 0);
    if (ar.branches == 1) for (int x = 1; x < kMaxBranches; ++x) CHECK(ar.direct[x].empty());
    // within a scene, a pass that depends on an earlier one runs in a later step
    for (size_t a = 0; a < np; ++a)
        for (size_t b = a + 1; b < np && ar.phase_scene[b] == ar.phase_scene[a]; ++b)
            if (conflict(acc[a], acc[b])) CHECK(step_of[b] > step_of[a]);
    // passes that share a step of a queue touch no common buffer
    for (size_t a = 0; a < np; ++a)
        for (size_t b = a + 1; b < np; ++b)
            if (queue_of[a] == queue_of[b] && step_of[a] == step_of[b] &&
                ar.phase_scene[a] != ar.phase_scene[b])
                CHECK(!conflict(acc[a], acc[b]));
    // queues run unordered: a buffer one queue writes is touched by no other
    std::vector<std::pair<const void *, int>> writers, users;
    for (size_t a = 0; a < np; ++a) {
        for (const void *p : acc[a].wr) writers.push_back({p, queue_of[a]});
        for (const void *p : acc[a].rd) users.push_back({p, queue_of[a]});
        for (const void *p : acc[a].wr) users.push_back({p, queue_of[a]});
    }
    std::sort(writers.begin(), writers.end());
    std::sort(users.begin(), users.end());
    for (auto &w : writers) {
        auto it = std::lower_bound(users.begin(), users.end(), std::make_pair(w.first, -1));
        for (; it != users.end() && it->first == w.first; ++it) CHECK(it->second == w.second);
    }
    // scenes of one slot run one after another, in disjoint steps; slots lie
    // inside the workspace without overlapping each other
    std::vector<int> lo(count, 1 << 30), hi(count, -1);
    for (size_t a = 0; a < np; ++a) {
        lo[ar.phase_scene[a]] = std::min(lo[ar.phase_scene[a]], step_of[a]);
        hi[ar.phase_scene[a]] = std::max(hi[ar.phase_scene[a]], step_of[a]);
    }
    std::vector<size_t> slot_size(ar.slot_base.size(), 0);
    for (int i = 0; i < count; ++i) {
        if (ar.scene_slot[i] < 0) continue;
        const Layout L = make_layout(sc[i].log2_size, sc[i].grad_fluence != nullptr);
        slot_size[ar.scene_slot[i]] = std::max(slot_size[ar.scene_slot[i]], L.total);
        for (int j = i + 1; j < count; ++j)
            if (ar.scene_slot[j] == ar.scene_slot[i]) CHECK(hi[i] < lo[j] || hi[j] < lo[i]);
    }
    std::vector<std::pair<size_t, size_t>> regions;
    for (size_t k = 0; k < slot_size.size(); ++k) regions.push_back({ar.slot_base[k], slot_size[k]});
    std::sort(regions.begin(), regions.end());
    size_t end = 0;
    for (auto &r : regions) {
        CHECK(r.first >= end);
        end = r.first + r.second;
    }
    CHECK(end <= ar.ws_bytes);
}

int main() {
    // ---- C ABI argument checks (no device call is reached) -----------------
    size_t f = 0, b = 0;
    CHECK(hrc_workspace_bytes(2, 0, &f, &b) == HRC_ERR_SHAPE);
    CHECK(hrc_workspace_bytes(13, 0, &f, &b) == HRC_ERR_SHAPE);
    CHECK(hrc_workspace_bytes(5, 0x8000u, &f, &b) == HRC_ERR_UNSUPPORTED);
    const unsigned fl[] = {0u, HRC_FLAG_HALF_INTERVALS, HRC_FLAG_QUADRANTS_1, HRC_FLAG_QUADRANTS_2,
                           HRC_FLAG_QUADRANTS_4, HRC_FLAG_BLUR};
    for (int N = HRC_MIN_LOG2; N <= HRC_MAX_LOG2; ++N) {
        for (unsigned x : fl) CHECK(hrc_workspace_bytes(N, x, &f, &b) == HRC_OK);
        for (int g : {1, 2, 4}) check_layout(make_layout(N, false, g), false);
        check_layout(make_layout(N, true), true);
    }
    char *p = fake(0), *ws = fake(1);
    float *fp = reinterpret_cast<float *>(fake(2));
    hrc_context *nctx = nullptr;
    CHECK(hrc_forward(nctx, 2, fp, fp, fp, ws, 1u << 30, nullptr, 0) == HRC_ERR_SHAPE);
    CHECK(hrc_forward(nctx, 5, fp + 1, fp, fp, ws, 1u << 30, nullptr, 0) == HRC_ERR_INVALID_ARG);
    CHECK(hrc_forward(nctx, 5, fp, fp, fp, ws, 1u << 30, nullptr, 0x8000u) == HRC_ERR_UNSUPPORTED);
    CHECK(hrc_forward(nctx, 5, fp, fp, fp, ws, 16, nullptr, 0) == HRC_ERR_WORKSPACE);
    CHECK(hrc_forward(nctx, 5, fp, fp, fp, ws, 1u << 30, nullptr, 0) == HRC_ERR_INVALID_ARG);
    CHECK(hrc_backward(nctx, 5, fp, fp, fp, fp, fp, ws, 1u << 30, nullptr, 0x8000u) ==
          HRC_ERR_UNSUPPORTED);
    CHECK(hrc_backward(nctx, 5, fp, fp, fp, fp, fp, ws, 1u << 30, nullptr,
                       HRC_FLAG_HALF_INTERVALS) == HRC_ERR_INVALID_ARG);  // no context
    for (int N = HRC_MIN_LOG2; N <= HRC_MAX_LOG2; ++N)
        check_layout(make_layout(N, true, 4, true), true, 4);  // the 16-bit reverse
    CHECK(hrc_backward(nctx, 5, fp, fp, fp, fp, fp, ws, 16, nullptr, 0) == HRC_ERR_WORKSPACE);
    CHECK(hrc_forward_static(nctx, 10, fp, fp, fp, nullptr, 0) == HRC_ERR_TOO_LARGE);
    CHECK(hrc_forward_static(nctx, 9, fp, fp, fp, nullptr, HRC_FLAG_VALIDATE) ==
          HRC_ERR_UNSUPPORTED);
    CHECK(hrc_forward_static(nctx, 9, fp, fp, fp, nullptr, 0) == HRC_ERR_INVALID_ARG);
    CHECK(hrc_multibounce_workspace_bytes(5, 0, 0, &f, &b) == HRC_ERR_INVALID_ARG);
    for (int st = 0; st >= -8; --st) CHECK(hrc_status_string((hrc_status)st) != nullptr);
    hrc_batch *bp = nullptr;
    hrc_scene one{};
    one.log2_size = 5;
    one.emission = one.sigma_t = fp;
    one.fluence = fp;
    CHECK(hrc_batch_plan(nctx, &one, 1, 0, nullptr, nullptr) == HRC_ERR_INVALID_ARG);
    CHECK(hrc_batch_plan(nctx, &one, 0, 0, nullptr, &bp) == HRC_ERR_INVALID_ARG);
    CHECK(hrc_batch_plan(nctx, &one, 1, 0x800u, nullptr, &bp) == HRC_ERR_UNSUPPORTED);
    CHECK(hrc_batch_plan(nctx, &one, 1, 0, nullptr, &bp) == HRC_ERR_INVALID_ARG);
    one.log2_size = 13;
    CHECK(hrc_batch_plan(nctx, &one, 1, 0, nullptr, &bp) == HRC_ERR_SHAPE);
    CHECK(hrc_batch_status(nullptr, nullptr) == HRC_ERR_INVALID_ARG);
    CHECK(hrc_batch_launch(nullptr, nullptr) == HRC_ERR_INVALID_ARG);
    hrc_destroy(nullptr);
    hrc_batch_destroy(nullptr);
    (void)p;

    // ---- the planner on fake scenes ----------------------------------------
    std::vector<hrc_scene> sc;
    const int sizes[] = {7, 10, 8, 9, 7, 10, 9, 8, 7, 8, 10, 9, 7, 9, 8, 10, 3, 4};
    for (int i = 0; i < (int)(sizeof(sizes) / sizeof(sizes[0])); ++i) {
        hrc_scene s{};
        s.log2_size = sizes[i];
        s.emission = reinterpret_cast<float *>(fake(100 + 8 * i));
        s.sigma_t = reinterpret_cast<float *>(fake(101 + 8 * i));
        s.fluence = reinterpret_cast<float *>(fake(102 + 8 * i));
        if (i % 5 != 3) {  // some scenes forward only
            s.grad_fluence = reinterpret_cast<float *>(fake(103 + 8 * i));
            s.grad_emission = reinterpret_cast<float *>(fake(104 + 8 * i));
            s.grad_sigma_t = reinterpret_cast<float *>(fake(105 + 8 * i));
        }
        sc.push_back(s);
    }
    int arrangements = 0;
    for (int nq : {1, 8})
        for (int slots : {0, 1, 2})
            for (int md : {HRC_MAX_LOG2 + 1, 10, 9})
                for (int quarters : {1, 4})
                    for (int target : {64, 2048})
                        for (int branches : {1, 2, 4}) {
                        if (md > HRC_MAX_LOG2 && branches > 1) continue;
                        Arrangement ar;
                        ar.min_direct = md;
                        ar.branches = branches;
                        ar.nqueues = nq;
                        ar.slots = slots;
                        ar.quarters = quarters;
                        ar.target = target;
                        arrange(ar, sc.data(), (int)sc.size(), fake(10000));
                        Arrangement sizes_only = ar;
                        arrange(sizes_only, sc.data(), (int)sc.size(), nullptr);
                        CHECK(sizes_only.ws_bytes == ar.ws_bytes);
                        check_arrangement(ar, sc);
                        ++arrangements;
                    }
    std::printf("host driver: %d arrangements checked, %d failures\n", arrangements, fails);
    return fails ? 1 : 0;
}
