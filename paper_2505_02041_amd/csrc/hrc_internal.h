// Internal declarations shared by the host API, the batch planner and the HIP
// kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// Opaque handle of the C ABI.
struct hrc_context {
    int device;
    int num_cus;
    float *env;    // device [4][kConeTable]: environment fluence per quadrant and cone
    int has_env;   // set by hrc_set_environment
    char *scratch; // device address of hrc_forward_static's scratch on this device
};

namespace hrc {

constexpr int kQuadrants = 4;
constexpr int kTracedLevels = 3;  // T_0..T_2 are traced directly (Section 4.2)
constexpr int kMaxLog2 = 12;
constexpr int kConeTable = (1 << (kMaxLog2 + 1)) - 1;  // sum over m <= 12 of 2^m

// Entries of T_n for one quadrant: (S >> n) columns x (2^n + 1) directions x S rows.
inline size_t t_level_entries(int N, int n) {
    size_t S = size_t(1) << N;
    return (S >> n) * ((size_t(1) << n) + 1) * S;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of every region inside a forward or backward workspace.
struct Layout {
    int N = 0;
    size_t S = 0;
    int group = 4;                       // quadrants whose pyramids are live at once
    size_t t_level[kMaxLog2 + 2] = {};   // T_n: `group` quadrants x t_level_entries float2
    size_t r_level[kMaxLog2 + 1] = {};   // R buffers: `group` quadrants x S^2 float each
    int r_count = 0;                     // 2 (forward ping-pong) or N (keeps every R_n)
    size_t aux = 0;                      // forward: one S^2 field (the gather before the blur)
    size_t dt_level[kMaxLog2 + 2] = {};  // backward: adjoint pyramid
    size_t dr_level[kMaxLog2 + 1] = {};  // backward: adjoint cascades
    size_t total = 0;
};

// Forward: pyramids of `group` quadrants (1, 2 or 4) at a time; backward: all 4.
// half: the forward's interval levels as 16-bit (L, T) pairs (4 bytes an entry).
// rgb (forward only): intervals (L_r, L_g, L_b, T) of 16 bytes, and the R
// levels and the spare field as three planes each.
Layout make_layout(int N, bool backward, int group = 4, bool half = false, bool rgb = false);

struct Ws {
    char *base;
    Layout L;
    float2 *T(int n) const { return reinterpret_cast<float2 *>(base + L.t_level[n]); }
    float2 *dT(int n) const { return reinterpret_cast<float2 *>(base + L.dt_level[n]); }
    float *R(int i) const { return reinterpret_cast<float *>(base + L.r_level[i]); }
    float *dR(int i) const { return reinterpret_cast<float *>(base + L.dr_level[i]); }
    float *Aux() const { return reinterpret_cast<float *>(base + L.aux); }
};

// ---- Arguments of each phase (one pass over one level of one scene) -------

// Forward passes run on a group of nq quadrants q0 .. q0+nq-1 whose buffers
// start at the pointers given (quadrant q0 first).
struct SeedArgs {
    const float *eps, *sig;
    float2 *T0, *T1, *T2;
    size_t e0, e1, e2;  // entries per quadrant of each level
    int N, q0, nq;
    int tile;           // image tile side: 32 standalone, 16 in the persistent kernel
    int first;          // first level written: 0, or 2 when the tail folds T_0 and T_1 itself
    int half;           // T levels stored as 16-bit (L, T) pairs (HRC_FLAG_HALF_INTERVALS)
};
// half: both levels stored as 16-bit (L, T) pairs (the pointers then address
// pairs of halves; the entry counts are unchanged)
struct UpArgs { const float2 *Tp; float2 *T; size_t ep, e; int N, n, nq; int half; };
// env (nullable): the environment's angular fluence per quadrant and cone,
// [4][kConeTable] with cone jj of level m at (2^m - 1) + jj, read for every
// angular fluence looked up outside the grid (and for R_N); NULL gives 0.
struct DownArgs {
    const float *Rn1;        // R_{n+1}; unused when n + 1 == N
    const float2 *Tn, *Tn1;  // T_n, T_{n+1}
    float *R;                // R_n
    size_t en, en1;
    int N, n, nq;
    const float *env;        // environment table (nullable)
    int q0;                  // absolute quadrant of the group's first solve
    int half;                // T levels stored as 16-bit (L, T) pairs
    int blk = 0;             // log2 of the direction block of the row order (0: column-major)
};
// The tail of the forward: levels 1 and 0 of the merge down, the gather and
// the sum over quadrants, from R_2 of the group's quadrants q0 .. q0+nq-1.
struct TailArgs {
    const float *eps, *sig;
    const float *R2;         // R_2, nq quadrants of S^2 floats (quadrant q0 first)
    float *out;              // F, [S][S]
    int N, q0, nq;
    int accumulate;          // add to out (the groups after the first) instead of storing
    const float *env;        // environment table (nullable)
    int tile;                // image tile side: 32 standalone, 16 in the persistent kernel
};
struct GatherAdjArgs { const float *dF; float *dR0; int N; };
struct DownAdjArgs {
    const float *dR;         // dR_n
    const float2 *Tn, *Tn1;
    float *dRn1;             // dR_{n+1}
    size_t en, en1;
    int N, n;
    int half;                // T levels stored as 16-bit (L, T) pairs
};
struct DTArgs {
    const float2 *Tn;        // T_n
    const float2 *dTn1;      // dT_{n+1} (when T_{n+1} is merged up from T_n)
    const float *dRn;        // dR_n
    const float *dRm;        // dR_{n-1}
    const float *Rn1;        // R_{n+1}
    const float *Rn;         // R_n
    float2 *dT;              // out: dT_n
    size_t en, en1;
    int N, n, has_up;
    const float *env;        // environment table (nullable), all four quadrants
    int half;                // T levels stored as 16-bit (L, T) pairs (dT stays FP32)
};
struct SeedAdjArgs {
    const float *eps, *sig;
    const float2 *dT0, *dT1, *dT2;
    size_t e0, e1, e2;
    float *dE, *dS;          // d eps, d sigma of the image [S][S]
    int N;
};

// Cross blur after the gather (Eq. 21) and its transpose: out = blur(F) with
// the opacity of each pixel alpha = 1 - exp(-sigma), neighbours further than
// `thr` in opacity (or outside the grid) ignored and the weights renormalised.
struct BlurArgs {
    const float *in;   // F (forward) or dLoss/d(blurred F) (adjoint)
    const float *sig;
    float *out;        // blurred F (forward) or dLoss/dF (adjoint)
    int N;
    float thr;
};

enum PhaseKind {
    PH_SEED = 0, PH_UP, PH_DOWN, PH_TAIL, PH_GATHER_ADJ,
    PH_DOWN_ADJ, PH_DT, PH_SEED_ADJ, PH_BLUR, PH_BLUR_ADJ,
    // the RGB solve (three radiance channels over one medium) and its reverse
    PH_SEED_RGB, PH_UP_RGB, PH_DOWN_RGB, PH_TAIL_RGB,
    PH_DOWN_ADJ_RGB, PH_DT_RGB, PH_SEED_ADJ_RGB, PH_KIND_COUNT
};

// One pass.  U = elements per thread of the elementwise phases (a tile covers
// 256*U consecutive outputs).
struct Phase {
    int kind = 0;
    int U = 1;
    int xblk = 0;  // log2 of the tile blocks dealt round-robin to the XCDs (0: contiguous eighths)
    union A {
        SeedArgs seed;
        UpArgs up;
        DownArgs down;
        TailArgs tail;
        GatherAdjArgs ga;
        DownAdjArgs da;
        DTArgs dt;
        SeedAdjArgs sa;
        BlurArgs bl;
        A() : dt{} {}
    } a;
};

// The phase list of one forward (and, with grads, backward) solve, in order.
// `U` gives elements per thread per phase kind (NULL = 1 everywhere).
struct SolveBuffers {
    const float *eps, *sig;
    float *F;
    const float *dF;
    float *dE, *dS;  // all three NULL: forward only
    int blur = 0;    // cross blur after the gather (forward) / its transpose first (reverse)
    const float *env = nullptr;  // environment table (hrc_context::env) or NULL
    int half = 0;    // interval levels stored as 16-bit pairs (the reverse's adjoints stay FP32)
};
// Opacity threshold of the cross blur (Eq. 21): |alpha_nb - alpha| above it ignores
// the neighbour.
constexpr float kBlurThreshold = 0.5f;
// keep_all_r: the reverse's layout, every level kept (forward down to R_1).
// recompute = false (with keep_all_r and a gradient): only the reverse, on
// the levels a kept forward left in the workspace.
int build_solve_phases(const Ws &w, const SolveBuffers &b, bool keep_all_r, const int *U,
                       Phase *out, int max_out, bool recompute = true);
// The passes of one RGB forward (all four quadrants at once): eps is [3][S][S],
// F is [3][S][S]; with blur, each plane is blurred by the one-channel pass.
int build_rgb_forward_phases(const Ws &w, const SolveBuffers &b, Phase *out, int max_out);
// The RGB solve in the reverse's layout: with recompute the forward down to R_1
// (then, given F, the tail and the blur), with a gradient the reverse.
int build_rgb_backward_phases(const Ws &w, const SolveBuffers &b, Phase *out, int max_out,
                              bool recompute);

unsigned phase_tiles(const Phase &p);
hipError_t upload_cone_table(const float *host_table);
// Launches one pass.  With events, they are recorded at the kernel's own start
// and end (a timed launch: no separate event packets between kernels).
hipError_t launch_phase(const Phase &p, hipStream_t s, hipEvent_t start = nullptr,
                        hipEvent_t stop = nullptr);
// Device tables of a planned batch.  The work is split over `nqueues` queues;
// with `xcd_local` each queue belongs to one XCD (accelerator complex die) and
// is served only by the blocks running there, which then see each other's
// stores in that XCD's L2 without writing the L2 back.  Queue q holds the
// segments [q_seg[q], q_seg[q+1]) and the steps [q_step[q], q_step[q+1]);
// segment i covers the queue's items [seg_start[i], seg_start[i+1]) (the last
// one up to q_items[q]) = the tiles of phase seg_phase[i], in step seg_step[i]
// (counted from the queue's first step); step_items[q_step[q] + t] counts the
// items of step t of queue q.
// The persistent kernel's blocks hold one or four 256-thread quarters
// (persistent_quarters(variant)), each running one tile; work is scheduled in
// groups of that many consecutive tiles of one phase (phases padded with empty
// tiles to whole groups).
constexpr int kMaxQuarters = 4;
constexpr int kMaxBranches = 4;  // graph branches of a batch's direct scenes
constexpr int kMaxQueues = 16;
struct BatchTables {
    const Phase *phases;
    const unsigned *seg_start;   // first group of each segment, counted within its queue
    const int *seg_phase;
    const int *seg_step;
    const unsigned *step_items;  // groups per step
    int nqueues;
    int xcd_local;               // queue q is served by the blocks of XCD q
    int q_seg[kMaxQueues + 1];
    int q_step[kMaxQueues + 1];
    unsigned q_items[kMaxQueues];
    unsigned chunk;              // groups a block claims at once
};
// Scheduler words, each in a cache line of its own (kSchedStride words apart):
// line 0 the error word (bits: 1 a dependency wait gave up, 2 a queue was left
// unfinished), line 1 the wait configuration (word 0: polls before a wait gives
// up, 0 for the default; word 1: groups added to what every wait needs, for
// failure tests), line 2 the count of blocks that have finished, then one claim
// counter per queue, then one completion count per step of each queue.  A
// launch clears everything from line 2 on; the error word and the
// configuration persist across launches.
constexpr unsigned kSchedStride = 32;
constexpr unsigned kSchedError = 0, kSchedConfig = 1, kSchedExit = 2, kSchedClaim = 3;
constexpr size_t sched_words(int nqueues, int total_steps) {
    return (size_t)kSchedStride * (kSchedClaim + nqueues + total_steps);
}
// Clears the per-launch scheduler words and launches the persistent kernel.
// Variants: 0 and 1 run 1024-thread blocks (four tiles side by side) with the
// full register budget or with 64 VGPRs (twice the resident blocks); 2 and 3
// run 256-thread blocks (one tile), likewise.
constexpr int kPersistentVariants = 4;
constexpr int persistent_quarters(int variant) { return variant < 2 ? 4 : 1; }
hipError_t launch_persistent(const BatchTables &t, unsigned *sched, int grid, int variant,
                             hipStream_t s);
hipError_t persistent_occupancy(int variant, int *blocks_per_cu);
// Writes the XCD of every block of a `grid`-block launch of `variant`'s block
// size to out[block] (the queue a block of the persistent kernel would serve).
hipError_t launch_xcd_probe(unsigned *out, int grid, int variant, hipStream_t s);
hipError_t launch_validate(const float *a, const float *b, size_t n, int *flag,
                           hipStream_t s);

// Several diffuse bounces: the next bounce's emission eps_0 + a sigma F / (2 pi)
// (isotropic in-scattering), and the reverse step of that update given dLoss/d
// eps_k = dE and the bounce's dLoss/d sigma = dS: d_eps += dE, d_sig += dS +
// a F_prev dE / (2 pi), d_alb += sigma F_prev dE / (2 pi), g = a sigma dE / (2 pi)
// (the previous bounce's dLoss/dF).  F_prev NULL: the first bounce (no source
// term; g untouched, d_alb untouched or, with assign, zero).  assign: overwrite
// the sums instead of adding.
hipError_t launch_scatter_source(const float *eps0, const float *sig, const float *alb,
                                 const float *F, float *out, size_t n, hipStream_t s);
hipError_t launch_scatter_adj(const float *dE, const float *dS, const float *F_prev,
                              const float *sig, const float *alb, float *g, float *d_eps,
                              float *d_sig, float *d_alb, size_t n, int assign, hipStream_t s);

constexpr int kMaxPhases = 8 * kMaxLog2 + 16;  // passes of one forward + backward solve

// RAII switch to a device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (ok && hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace hrc
