// Host side of the C ABI: argument checks, workspace layout, context, and the
// per-level launch sequence of Algorithm 1 (forward) and of its reverse.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <vector>

#include "../../include/hrc.h"
#include "hrc_internal.h"

namespace hrc {

Layout make_layout(int N, bool backward, int group, bool half, bool rgb) {
    Layout L;
    L.N = N;
    L.S = size_t(1) << N;
    L.group = backward ? kQuadrants : group;
    const size_t SS = L.S * L.S;
    const size_t planes = rgb ? 3 : 1;
    size_t off = 256;  // first 256 bytes: scratch flag for HRC_FLAG_VALIDATE
    // the forward's tail folds T_0 and T_1 itself (only the reverse stores
    // them), and the merge down builds what it reads of T_N itself
    const size_t iv_bytes = rgb    ? (half ? 4 * sizeof(uint16_t) : sizeof(float4))
                            : half ? 2 * sizeof(uint16_t)
                                   : sizeof(float2);
    for (int n = backward ? 0 : kTracedLevels - 1; n < N; ++n) {
        L.t_level[n] = off;
        off += align256(L.group * t_level_entries(N, n) * iv_bytes);
    }
    L.r_count = backward ? N : 2;
    for (int i = 0; i < L.r_count; ++i) {
        L.r_level[i] = off;
        off += align256(planes * L.group * SS * sizeof(float));
    }
    if (!backward) {
        L.aux = off;
        off += align256(planes * SS * sizeof(float));
    }
    if (backward) {
        for (int n = 0; n <= N; ++n) {
            L.dt_level[n] = off;
            off += align256(kQuadrants * t_level_entries(N, n) * (rgb ? sizeof(float4) : sizeof(float2)));
        }
        for (int i = 0; i < N; ++i) {
            L.dr_level[i] = off;
            off += align256(planes * kQuadrants * SS * sizeof(float));
        }
    }
    L.total = off;
    return L;
}

// Flags hrc_forward, hrc_backward and hrc_workspace_bytes accept; the bounce
// calls and the profile take those of kSolveFlags.
static constexpr unsigned kSolveFlags =
    HRC_FLAG_VALIDATE | HRC_FLAG_QUADRANTS_MASK | HRC_FLAG_BLUR;
static constexpr unsigned kForwardFlags = kSolveFlags | HRC_FLAG_HALF_INTERVALS;
// hrc_forward and the workspace query also take HRC_FLAG_KEEP_PYRAMID,
// hrc_backward HRC_FLAG_REUSE_PYRAMID.
static constexpr unsigned kKeepFlags = kForwardFlags | HRC_FLAG_KEEP_PYRAMID;
static constexpr unsigned kReuseFlags = kForwardFlags | HRC_FLAG_REUSE_PYRAMID;

// HRC_FLAG_KEEP_PYRAMID computes all four quadrants at once.
static bool keep_group_ok(unsigned flags) {
    const unsigned g = flags & HRC_FLAG_QUADRANTS_MASK;
    return !(flags & HRC_FLAG_KEEP_PYRAMID) || g == 0 || g == HRC_FLAG_QUADRANTS_4;
}

// Quadrant group of a forward: from the flags, else all four at once.
static int forward_group(int N, unsigned flags) {
    switch ((flags & HRC_FLAG_QUADRANTS_MASK) >> 4) {
        case 1: return 1;
        case 2: return 2;
        case 3: return 4;
        default: return 4;  // the fastest at every size measured (1024^2 .. 4096^2)
    }
}

// A_m(jj) of Eq. 13 in double precision, rounded once to float.
static void cone_table(float *out) {
    for (int m = 0; m <= kMaxLog2; ++m) {
        const double a = double(1 << m);
        for (int jj = 0; jj < (1 << m); ++jj) {
            double hi = atan2(2.0 * (jj + 1) - a, a);
            double lo = atan2(2.0 * jj - a, a);
            out[(1 << m) - 1 + jj] = float(hi - lo);
        }
    }
}

// Environment fluence per quadrant and cone (the footnote to Section 4.2): for
// quadrant q, level m <= HRC_MAX_LOG2 and cone jj, A_m(jj) times the radiance of
// the map in the world direction of the cone's centre v_m(jj + 1/2), the map
// being K samples at angles 2 pi k / K from +x (columns) towards +y (rows),
// nearest sample (halfway: the next one counter-clockwise).  Quadrant frames:
// +x (u, w) = (c, r), -x (S-1-c, r), +y (r, c), -y (S-1-r, c).
static void environment_table(const float *radiance, int K, float *out) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int q = 0; q < kQuadrants; ++q) {
        for (int m = 0; m <= kMaxLog2; ++m) {
            const double a = double(1 << m);
            for (int jj = 0; jj < (1 << m); ++jj) {
                const double du = a, dw = 2.0 * jj + 1.0 - a;
                double dc, dr;
                switch (q) {
                    case 0: dc = du; dr = dw; break;
                    case 1: dc = -du; dr = dw; break;
                    case 2: dc = dw; dr = du; break;
                    default: dc = dw; dr = -du; break;
                }
                long k = (long)floor(atan2(dr, dc) * K / two_pi + 0.5) % K;
                if (k < 0) k += K;
                const double A = atan2(2.0 * (jj + 1) - a, a) - atan2(2.0 * jj - a, a);
                out[(size_t)q * kConeTable + (1 << m) - 1 + jj] = float(A * radiance[k]);
            }
        }
    }
}

// Scratch of hrc_forward_static: the FP32 forward workspace of the largest
// grid it takes (2^9 per side, all four quadrants at once: 72,319,232 bytes),
// in device memory every device the library runs on holds until the process
// ends.  Host code never passes the array's name to a kernel or a copy: it
// uses the device address hrc_create looked up (hrc_context::scratch).
constexpr int kStaticMaxLog2 = 9;
constexpr size_t kStaticScratchBytes = size_t(69) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

static bool aligned16(const void *p) { return p && (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

static hrc_status check_shape(int log2_size) {
    return (log2_size < HRC_MIN_LOG2 || log2_size > HRC_MAX_LOG2) ? HRC_ERR_SHAPE : HRC_OK;
}

static int pick_u(const int *U, int kind) { return U ? (U[kind] > 0 ? U[kind] : 1) : 1; }

// The passes of one solve in execution order (Algorithm 1 for the four
// quadrants at once, then, with gradients, its reverse).  R levels either all
// kept (R(n) = R_n, needed by the reverse) or alternating in two buffers.
// Tile order of the elementwise passes from 1024^2 up: blocks of tiles dealt
// round robin to the XCDs (log2 of the block; 0 below, where the contiguous
// eighths were as fast or faster).  For the adjoints, blocks of 2^(N-6) were
// as fast as 2^(N-5) and the larger ones split fewer shared rows across XCDs.  Measured against contiguous eighths: the
// forward 2-7%, the RGB forward 4% and the reverse 3-9% faster at 1024^2 ..
// 4096^2; the same results, since only the order of the tiles changes.
static int tile_order(int N, int kind) {
    if (N < 10) return 0;
    switch (kind) {
        case PH_UP:
        case PH_UP_RGB: return 7;
        case PH_DOWN:
        case PH_DOWN_RGB: return 9;
        case PH_DOWN_ADJ:
        case PH_DOWN_ADJ_RGB:
        case PH_DT:
        case PH_DT_RGB: return N - 5;
        default: return 0;
    }
}

int build_solve_phases(const Ws &w, const SolveBuffers &b, bool keep_all_r, const int *U,
                       Phase *out, int max_out, bool recompute) {
    const int N = w.L.N;
    int np = 0;
    auto add = [&](Phase p) {
        p.xblk = tile_order(N, p.kind);
        if (np < max_out) out[np] = p;
        ++np;
    };
    Phase p;
    // Algorithm 1 for `group` quadrants at a time; each group reuses the same
    // pyramid buffers.  The merge down runs to level 2 (forward: the tail
    // builds levels 1 and 0 on chip) or, when every level is kept for the
    // reverse, to level 1, the last one the reverse reads; then the tail adds
    // the group's quadrants to F.  With the blur, the gather goes first to a
    // buffer that is free by then: the forward's spare field, or (every level
    // kept) dR_0, which the reverse writes only later.
    const int G = w.L.group;
    float *gathered = b.blur ? (keep_all_r ? w.dR(0) : w.Aux()) : b.F;
    for (int q0 = 0; recompute && q0 < kQuadrants; q0 += G) {
        p = Phase();
        p.kind = PH_SEED;
        p.a.seed = SeedArgs{b.eps,
                            b.sig,
                            keep_all_r ? w.T(0) : nullptr,
                            keep_all_r ? w.T(1) : nullptr,
                            w.T(2),
                            t_level_entries(N, 0),
                            t_level_entries(N, 1),
                            t_level_entries(N, 2),
                            N,
                            q0,
                            G,
                            32,
                            keep_all_r ? 0 : kTracedLevels - 1,
                            b.half};
        add(p);
        for (int n = kTracedLevels; n < N; ++n) {
            p = Phase();
            p.kind = PH_UP;
            p.U = pick_u(U, PH_UP);
            p.a.up = UpArgs{w.T(n - 1), w.T(n), t_level_entries(N, n - 1), t_level_entries(N, n),
                            N, n, G, b.half};
            add(p);
        }
        int cur = -1;
        const int n_last = keep_all_r ? 1 : 2;
        for (int n = N - 1; n >= n_last; --n) {
            const int o = keep_all_r ? n : (cur == 0 ? 1 : 0);
            p = Phase();
            p.kind = PH_DOWN;
            p.U = pick_u(U, PH_DOWN);
            p.a.down = DownArgs{(n + 1 < N) ? w.R(cur) : nullptr, w.T(n), w.T(n + 1), w.R(o),
                                t_level_entries(N, n), t_level_entries(N, n + 1), N, n, G,
                                b.env, q0, b.half};
            // the top three levels (at most eight probe columns) in blocks of
            // 32 directions: the columns that share R_{n+1} and T rows then run
            // on one XCD (2-8% faster at these levels, same results)
            if (N - n <= 3) p.a.down.blk = n < 5 ? n : 5;
            add(p);
            cur = o;
        }
        if (b.F) {
            p = Phase();
            p.kind = PH_TAIL;
            p.a.tail = TailArgs{b.eps, b.sig, keep_all_r ? w.R(2) : w.R(cur), gathered,
                                N, q0, G, q0 > 0 ? 1 : 0, b.env, 32};
            add(p);
        }
    }
    if (recompute && b.F && b.blur) {
        p = Phase();
        p.kind = PH_BLUR;
        p.a.bl = BlurArgs{gathered, b.sig, b.F, N, kBlurThreshold};
        add(p);
    }
    if (b.dF) {
        // with the blur, its transpose first, into R_0's buffer (neither the
        // kept forward nor the reverse uses R_0)
        const float *dgathered = b.dF;
        if (b.blur) {
            p = Phase();
            p.kind = PH_BLUR_ADJ;
            p.a.bl = BlurArgs{b.dF, b.sig, w.R(0), N, kBlurThreshold};
            add(p);
            dgathered = w.R(0);
        }
        p = Phase();
        p.kind = PH_GATHER_ADJ;
        p.a.ga = GatherAdjArgs{dgathered, w.dR(0), N};
        add(p);
        for (int n = 0; n + 1 < N; ++n) {
            p = Phase();
            p.kind = PH_DOWN_ADJ;
            p.U = pick_u(U, PH_DOWN_ADJ);
            p.a.da = DownAdjArgs{w.dR(n), w.T(n), w.T(n + 1), w.dR(n + 1), t_level_entries(N, n),
                                 t_level_entries(N, n + 1), N, n, b.half};
            add(p);
        }
        for (int n = N; n >= 0; --n) {
            p = Phase();
            p.kind = PH_DT;
            p.U = pick_u(U, PH_DT);
            DTArgs d{};
            d.Tn = w.T(n);
            d.has_up = (n + 1 <= N && n + 1 >= kTracedLevels) ? 1 : 0;
            d.dTn1 = d.has_up ? w.dT(n + 1) : nullptr;
            d.dRn = n < N ? w.dR(n) : nullptr;
            d.dRm = n >= 1 ? w.dR(n - 1) : nullptr;
            d.Rn1 = (n + 1 < N) ? w.R(n + 1) : nullptr;
            d.Rn = n < N ? w.R(n) : nullptr;
            d.dT = w.dT(n);
            d.en = t_level_entries(N, n);
            d.en1 = n + 1 <= N ? t_level_entries(N, n + 1) : 0;
            d.N = N;
            d.env = b.env;
            d.n = n;
            d.half = b.half;
            p.a.dt = d;
            add(p);
        }
        p = Phase();
        p.kind = PH_SEED_ADJ;
        p.a.sa = SeedAdjArgs{b.eps, b.sig, w.dT(0), w.dT(1), w.dT(2), t_level_entries(N, 0),
                             t_level_entries(N, 1), t_level_entries(N, 2), b.dE, b.dS, N};
        add(p);
    }
    return np;
}

int build_rgb_forward_phases(const Ws &w, const SolveBuffers &b, Phase *out, int max_out) {
    const int N = w.L.N;
    const size_t SS = w.L.S * w.L.S;
    int np = 0;
    auto add = [&](Phase p) {
        p.xblk = tile_order(N, p.kind);
        if (np < max_out) out[np] = p;
        ++np;
    };
    Phase p;
    float *gathered = b.blur ? w.Aux() : b.F;
    p.kind = PH_SEED_RGB;
    p.a.seed = SeedArgs{b.eps, b.sig, nullptr, nullptr, w.T(2), t_level_entries(N, 0),
                        t_level_entries(N, 1), t_level_entries(N, 2), N, 0, kQuadrants, 16,
                        kTracedLevels - 1, b.half};
    add(p);
    for (int n = kTracedLevels; n < N; ++n) {
        p = Phase();
        p.kind = PH_UP_RGB;
        p.a.up = UpArgs{w.T(n - 1), w.T(n), t_level_entries(N, n - 1), t_level_entries(N, n), N, n,
                        kQuadrants, b.half};
        add(p);
    }
    int cur = -1;
    for (int n = N - 1; n >= 2; --n) {
        const int o = cur == 0 ? 1 : 0;
        p = Phase();
        p.kind = PH_DOWN_RGB;
        p.a.down = DownArgs{(n + 1 < N) ? w.R(cur) : nullptr, w.T(n), w.T(n + 1), w.R(o),
                            t_level_entries(N, n), t_level_entries(N, n + 1), N, n, kQuadrants,
                            nullptr, 0, b.half};
        add(p);
        cur = o;
    }
    p = Phase();
    p.kind = PH_TAIL_RGB;
    p.a.tail = TailArgs{b.eps, b.sig, w.R(cur), gathered, N, 0, kQuadrants, 0, nullptr, 16};
    add(p);
    if (b.blur) {
        for (int c = 0; c < 3; ++c) {
            p = Phase();
            p.kind = PH_BLUR;
            p.a.bl = BlurArgs{gathered + c * SS, b.sig, b.F + c * SS, N, kBlurThreshold};
            add(p);
        }
    }
    return np;
}

// The RGB solve in the reverse's layout (every level kept, three planes per
// cascade level, float4 intervals and adjoints): with recompute, the forward
// down to R_1 (and, given F, the tail and the blur); with a gradient, the
// reverse.  Mirrors build_solve_phases for all four quadrants at once.
int build_rgb_backward_phases(const Ws &w, const SolveBuffers &b, Phase *out, int max_out,
                              bool recompute) {
    const int N = w.L.N;
    const size_t SS = w.L.S * w.L.S, plane = kQuadrants * SS;
    int np = 0;
    auto add = [&](Phase p) {
        p.xblk = tile_order(N, p.kind);
        if (np < max_out) out[np] = p;
        ++np;
    };
    Phase p;
    // the gather before the blur goes to dR_0, which the reverse writes only later
    float *gathered = b.blur ? w.dR(0) : b.F;
    if (recompute) {
        p.kind = PH_SEED_RGB;
        p.a.seed = SeedArgs{b.eps, b.sig, w.T(0), w.T(1), w.T(2), t_level_entries(N, 0),
                            t_level_entries(N, 1), t_level_entries(N, 2), N, 0, kQuadrants, 16, 0,
                            b.half};
        add(p);
        for (int n = kTracedLevels; n < N; ++n) {
            p = Phase();
            p.kind = PH_UP_RGB;
            p.a.up = UpArgs{w.T(n - 1), w.T(n), t_level_entries(N, n - 1), t_level_entries(N, n), N,
                            n, kQuadrants, b.half};
            add(p);
        }
        for (int n = N - 1; n >= 1; --n) {
            p = Phase();
            p.kind = PH_DOWN_RGB;
            p.a.down = DownArgs{(n + 1 < N) ? w.R(n + 1) : nullptr, w.T(n), w.T(n + 1), w.R(n),
                                t_level_entries(N, n), t_level_entries(N, n + 1), N, n, kQuadrants,
                                nullptr, 0, b.half};
            add(p);
        }
        if (b.F) {
            p = Phase();
            p.kind = PH_TAIL_RGB;
            p.a.tail = TailArgs{b.eps, b.sig, w.R(2), gathered, N, 0, kQuadrants, 0, nullptr, 16};
            add(p);
            if (b.blur) {
                for (int c = 0; c < 3; ++c) {
                    p = Phase();
                    p.kind = PH_BLUR;
                    p.a.bl = BlurArgs{gathered + c * SS, b.sig, b.F + c * SS, N, kBlurThreshold};
                    add(p);
                }
            }
        }
    }
    if (b.dF) {
        // with the blur, its transpose per channel first, into R_0's buffer
        const float *dgathered = b.dF;
        if (b.blur) {
            for (int c = 0; c < 3; ++c) {
                p = Phase();
                p.kind = PH_BLUR_ADJ;
                p.a.bl = BlurArgs{b.dF + c * SS, b.sig, w.R(0) + c * SS, N, kBlurThreshold};
                add(p);
            }
            dgathered = w.R(0);
        }
        for (int c = 0; c < 3; ++c) {
            p = Phase();
            p.kind = PH_GATHER_ADJ;
            p.a.ga = GatherAdjArgs{dgathered + c * SS, w.dR(0) + c * plane, N};
            add(p);
        }
        for (int n = 0; n + 1 < N; ++n) {
            p = Phase();
            p.kind = PH_DOWN_ADJ_RGB;
            p.a.da = DownAdjArgs{w.dR(n), w.T(n), w.T(n + 1), w.dR(n + 1), t_level_entries(N, n),
                                 t_level_entries(N, n + 1), N, n, b.half};
            add(p);
        }
        for (int n = N; n >= 0; --n) {
            p = Phase();
            p.kind = PH_DT_RGB;
            DTArgs d{};
            d.Tn = w.T(n);
            d.has_up = (n + 1 <= N && n + 1 >= kTracedLevels) ? 1 : 0;
            d.dTn1 = d.has_up ? w.dT(n + 1) : nullptr;
            d.dRn = n < N ? w.dR(n) : nullptr;
            d.dRm = n >= 1 ? w.dR(n - 1) : nullptr;
            d.Rn1 = (n + 1 < N) ? w.R(n + 1) : nullptr;
            d.Rn = n < N ? w.R(n) : nullptr;
            d.dT = w.dT(n);
            d.en = t_level_entries(N, n);
            d.en1 = n + 1 <= N ? t_level_entries(N, n + 1) : 0;
            d.N = N;
            d.n = n;
            d.half = b.half;
            p.a.dt = d;
            add(p);
        }
        p = Phase();
        p.kind = PH_SEED_ADJ_RGB;
        p.a.sa = SeedAdjArgs{b.eps, b.sig, w.dT(0), w.dT(1), w.dT(2), t_level_entries(N, 0),
                             t_level_entries(N, 1), t_level_entries(N, 2), b.dE, b.dS, N};
        add(p);
    }
    return np;
}

static hrc_status run_phases(const Phase *ph, int np, hipStream_t s) {
    for (int i = 0; i < np; ++i)
        if (launch_phase(ph[i], s) != hipSuccess) return HRC_ERR_HIP;
    return HRC_OK;
}

static hrc_status validate_inputs(const Ws &w, const float *eps, const float *sig,
                                  hipStream_t s) {
    int *flag = reinterpret_cast<int *>(w.base);
    int host = 0;
    if (hipMemsetAsync(flag, 0, sizeof(int), s) != hipSuccess) return HRC_ERR_HIP;
    if (launch_validate(eps, sig, w.L.S * w.L.S, flag, s) != hipSuccess) return HRC_ERR_HIP;
    if (hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        return HRC_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return HRC_ERR_HIP;
    return host ? HRC_ERR_INPUT : HRC_OK;
}

}  // namespace hrc

using namespace hrc;

extern "C" {

const char *hrc_status_string(hrc_status s) {
    switch (s) {
        case HRC_OK: return "HRC_OK";
        case HRC_ERR_INVALID_ARG: return "HRC_ERR_INVALID_ARG: NULL or misaligned pointer, NULL context or bad count";
        case HRC_ERR_SHAPE: return "HRC_ERR_SHAPE: log2_size outside [3, 12]";
        case HRC_ERR_WORKSPACE: return "HRC_ERR_WORKSPACE: workspace smaller than hrc_workspace_bytes";
        case HRC_ERR_HIP: return "HRC_ERR_HIP: a HIP runtime call or kernel launch failed";
        case HRC_ERR_UNSUPPORTED: return "HRC_ERR_UNSUPPORTED: unknown flag bits, or a flag this call does not take";
        case HRC_ERR_INPUT: return "HRC_ERR_INPUT: negative or non-finite emission or attenuation";
        case HRC_ERR_TIMEOUT: return "HRC_ERR_TIMEOUT: a dependency wait of the batch gave up; that launch's results are incomplete";
        case HRC_ERR_TOO_LARGE: return "HRC_ERR_TOO_LARGE: grid larger than hrc_forward_static's scratch holds (log2_size <= 9)";
    }
    return "HRC: unknown status";
}

hrc_status hrc_workspace_bytes(int log2_size, unsigned flags, size_t *forward_bytes,
                               size_t *backward_bytes) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if ((flags & ~(kKeepFlags | HRC_FLAG_REUSE_PYRAMID)) || !keep_group_ok(flags))
        return HRC_ERR_UNSUPPORTED;
    const bool keep = (flags & HRC_FLAG_KEEP_PYRAMID) != 0;
    if (forward_bytes)
        *forward_bytes = make_layout(log2_size, keep, forward_group(log2_size, flags),
                                     (flags & HRC_FLAG_HALF_INTERVALS) != 0)
                             .total;
    if (backward_bytes)
        *backward_bytes =
            make_layout(log2_size, true, 4, (flags & HRC_FLAG_HALF_INTERVALS) != 0).total;
    return HRC_OK;
}

hrc_status hrc_create(int device, hrc_context **out) {
    if (!out) return HRC_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return HRC_ERR_HIP;
    DeviceGuard g(device);
    if (!g.ok) return HRC_ERR_HIP;
    std::vector<float> table(kConeTable);
    cone_table(table.data());
    if (upload_cone_table(table.data()) != hipSuccess) return HRC_ERR_HIP;
    // the device address of hrc_forward_static's scratch on this device (each
    // device holds its own copy of the array)
    void *scr = nullptr;
    if (hipGetSymbolAddress(&scr, HIP_SYMBOL(scratch)) != hipSuccess || !scr) return HRC_ERR_HIP;
    hrc_context *ctx = static_cast<hrc_context *>(calloc(1, sizeof(hrc_context)));
    if (!ctx) return HRC_ERR_HIP;
    ctx->device = device;
    ctx->scratch = static_cast<char *>(scr);
    hipDeviceProp_t prop;
    ctx->num_cus = (hipGetDeviceProperties(&prop, device) == hipSuccess) ? prop.multiProcessorCount : 256;
    *out = ctx;
    return HRC_OK;
}

void hrc_destroy(hrc_context *ctx) {
    if (!ctx) return;
    if (ctx->env) {
        DeviceGuard g(ctx->device);
        (void)hipFree(ctx->env);
    }
    free(ctx);
}

hrc_status hrc_set_environment(hrc_context *ctx, const float *radiance, int samples) {
    if (!ctx || samples < 0 || (samples > 0 && !radiance)) return HRC_ERR_INVALID_ARG;
    for (int k = 0; k < samples; ++k)
        if (!std::isfinite(radiance[k])) return HRC_ERR_INPUT;
    if (samples == 0) {
        ctx->has_env = 0;
        return HRC_OK;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    const size_t bytes = sizeof(float) * kQuadrants * kConeTable;
    if (!ctx->env && hipMalloc(&ctx->env, bytes) != hipSuccess) {
        ctx->env = nullptr;
        return HRC_ERR_HIP;
    }
    std::vector<float> table((size_t)kQuadrants * kConeTable);
    environment_table(radiance, samples, table.data());
    if (hipMemcpy(ctx->env, table.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
        return HRC_ERR_HIP;
    ctx->has_env = 1;
    return HRC_OK;
}

hrc_status hrc_forward(hrc_context *ctx, int log2_size, const float *emission,
                       const float *sigma_t, float *fluence, void *workspace,
                       size_t workspace_bytes, void *stream, unsigned flags) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (!aligned16(emission) || !aligned16(sigma_t) || !aligned16(fluence) ||
        !aligned16(workspace))
        return HRC_ERR_INVALID_ARG;
    if ((flags & ~kKeepFlags) || !keep_group_ok(flags)) return HRC_ERR_UNSUPPORTED;
    const bool half = (flags & HRC_FLAG_HALF_INTERVALS) != 0;
    const bool keep = (flags & HRC_FLAG_KEEP_PYRAMID) != 0;
    // with KEEP: the reverse's layout, every level the reverse reads kept
    Layout L = make_layout(log2_size, keep, forward_group(log2_size, flags), half);
    if (workspace_bytes < L.total) return HRC_ERR_WORKSPACE;
    if (!ctx) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ws w{static_cast<char *>(workspace), L};
    if (flags & HRC_FLAG_VALIDATE) {
        st = validate_inputs(w, emission, sigma_t, s);
        if (st != HRC_OK) return st;
    }
    Phase ph[kMaxPhases];
    SolveBuffers b{emission, sigma_t, fluence, nullptr, nullptr, nullptr,
                   (flags & HRC_FLAG_BLUR) ? 1 : 0, ctx->has_env ? ctx->env : nullptr,
                   half ? 1 : 0};
    int np = build_solve_phases(w, b, keep, nullptr, ph, kMaxPhases);
    return run_phases(ph, np, s);
}

hrc_status hrc_forward_static(hrc_context *ctx, int log2_size, const float *emission,
                              const float *sigma_t, float *fluence, void *stream,
                              unsigned flags) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (!aligned16(emission) || !aligned16(sigma_t) || !aligned16(fluence))
        return HRC_ERR_INVALID_ARG;
    if (flags & ~(kForwardFlags & ~HRC_FLAG_VALIDATE)) return HRC_ERR_UNSUPPORTED;
    if (log2_size > kStaticMaxLog2) return HRC_ERR_TOO_LARGE;
    const bool half = (flags & HRC_FLAG_HALF_INTERVALS) != 0;
    Layout L = make_layout(log2_size, false, forward_group(log2_size, flags), half);
    if (L.total > kStaticScratchBytes) return HRC_ERR_TOO_LARGE;
    if (!ctx || !ctx->scratch) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    // the same passes and launch shapes as hrc_forward, on the scratch
    Ws w{ctx->scratch, L};
    Phase ph[kMaxPhases];
    SolveBuffers b{emission, sigma_t, fluence, nullptr, nullptr, nullptr,
                   (flags & HRC_FLAG_BLUR) ? 1 : 0, ctx->has_env ? ctx->env : nullptr,
                   half ? 1 : 0};
    int np = build_solve_phases(w, b, false, nullptr, ph, kMaxPhases);
    return run_phases(ph, np, static_cast<hipStream_t>(stream));
}

hrc_status hrc_backward(hrc_context *ctx, int log2_size, const float *emission,
                        const float *sigma_t, const float *grad_fluence, float *grad_emission,
                        float *grad_sigma_t, void *workspace, size_t workspace_bytes,
                        void *stream, unsigned flags) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (!aligned16(emission) || !aligned16(sigma_t) || !aligned16(grad_fluence) ||
        !aligned16(grad_emission) || !aligned16(grad_sigma_t) || !aligned16(workspace))
        return HRC_ERR_INVALID_ARG;
    if (flags & ~kReuseFlags) return HRC_ERR_UNSUPPORTED;
    const bool half = (flags & HRC_FLAG_HALF_INTERVALS) != 0;
    const bool reuse = (flags & HRC_FLAG_REUSE_PYRAMID) != 0;
    Layout L = make_layout(log2_size, true, 4, half);
    if (workspace_bytes < L.total) return HRC_ERR_WORKSPACE;
    if (!ctx) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ws w{static_cast<char *>(workspace), L};
    if (flags & HRC_FLAG_VALIDATE) {
        st = validate_inputs(w, emission, sigma_t, s);
        if (st != HRC_OK) return st;
    }
    Phase ph[kMaxPhases];
    SolveBuffers b{emission, sigma_t, nullptr, grad_fluence, grad_emission, grad_sigma_t,
                   (flags & HRC_FLAG_BLUR) ? 1 : 0, ctx->has_env ? ctx->env : nullptr,
                   half ? 1 : 0};
    int np = build_solve_phases(w, b, true, nullptr, ph, kMaxPhases, !reuse);
    return run_phases(ph, np, s);
}

// ---- three radiance channels (RGB) over one medium ---------------------------

static constexpr unsigned kRgbFlags = HRC_FLAG_VALIDATE | HRC_FLAG_BLUR | HRC_FLAG_HALF_INTERVALS;
// hrc_forward_rgb also takes HRC_FLAG_KEEP_PYRAMID, hrc_backward_rgb
// HRC_FLAG_REUSE_PYRAMID; the workspace query takes both.
static constexpr unsigned kRgbForwardFlags = kRgbFlags | HRC_FLAG_KEEP_PYRAMID;
static constexpr unsigned kRgbBackwardFlags = kRgbFlags | HRC_FLAG_REUSE_PYRAMID;

hrc_status hrc_workspace_bytes_rgb(int log2_size, unsigned flags, size_t *forward_bytes,
                                   size_t *backward_bytes) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (flags & ~(kRgbForwardFlags | HRC_FLAG_REUSE_PYRAMID)) return HRC_ERR_UNSUPPORTED;
    const bool keep = (flags & HRC_FLAG_KEEP_PYRAMID) != 0;
    const bool half = (flags & HRC_FLAG_HALF_INTERVALS) != 0;
    if (forward_bytes) *forward_bytes = make_layout(log2_size, keep, 4, half, true).total;
    if (backward_bytes) *backward_bytes = make_layout(log2_size, true, 4, half, true).total;
    return HRC_OK;
}

static hrc_status validate_rgb(const Ws &w, const float *emission, const float *sigma_t,
                               hipStream_t s) {
    const size_t SS = w.L.S * w.L.S;
    hrc_status st = validate_inputs(w, emission, emission + SS, s);
    if (st == HRC_OK) st = validate_inputs(w, emission + 2 * SS, sigma_t, s);
    return st;
}

hrc_status hrc_forward_rgb(hrc_context *ctx, int log2_size, const float *emission,
                           const float *sigma_t, float *fluence, void *workspace,
                           size_t workspace_bytes, void *stream, unsigned flags) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (!aligned16(emission) || !aligned16(sigma_t) || !aligned16(fluence) ||
        !aligned16(workspace))
        return HRC_ERR_INVALID_ARG;
    if (flags & ~kRgbForwardFlags) return HRC_ERR_UNSUPPORTED;
    const bool half = (flags & HRC_FLAG_HALF_INTERVALS) != 0;
    const bool keep = (flags & HRC_FLAG_KEEP_PYRAMID) != 0;
    Layout L = make_layout(log2_size, keep, 4, half, true);
    if (workspace_bytes < L.total) return HRC_ERR_WORKSPACE;
    if (!ctx) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ws w{static_cast<char *>(workspace), L};
    if (flags & HRC_FLAG_VALIDATE) {
        st = validate_rgb(w, emission, sigma_t, s);
        if (st != HRC_OK) return st;
    }
    Phase ph[kMaxPhases];
    SolveBuffers b{emission, sigma_t, fluence, nullptr, nullptr, nullptr,
                   (flags & HRC_FLAG_BLUR) ? 1 : 0, nullptr, half ? 1 : 0};
    int np = keep ? build_rgb_backward_phases(w, b, ph, kMaxPhases, true)
                  : build_rgb_forward_phases(w, b, ph, kMaxPhases);
    return run_phases(ph, np, s);
}

hrc_status hrc_backward_rgb(hrc_context *ctx, int log2_size, const float *emission,
                            const float *sigma_t, const float *grad_fluence,
                            float *grad_emission, float *grad_sigma_t, void *workspace,
                            size_t workspace_bytes, void *stream, unsigned flags) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (!aligned16(emission) || !aligned16(sigma_t) || !aligned16(grad_fluence) ||
        !aligned16(grad_emission) || !aligned16(grad_sigma_t) || !aligned16(workspace))
        return HRC_ERR_INVALID_ARG;
    if (flags & ~kRgbBackwardFlags) return HRC_ERR_UNSUPPORTED;
    const bool half = (flags & HRC_FLAG_HALF_INTERVALS) != 0;
    const Layout L = make_layout(log2_size, true, 4, half, true);
    if (workspace_bytes < L.total) return HRC_ERR_WORKSPACE;
    if (!ctx) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ws w{static_cast<char *>(workspace), L};
    if (flags & HRC_FLAG_VALIDATE) {
        st = validate_rgb(w, emission, sigma_t, s);
        if (st != HRC_OK) return st;
    }
    Phase ph[kMaxPhases];
    SolveBuffers b{emission, sigma_t, nullptr, grad_fluence, grad_emission, grad_sigma_t,
                   (flags & HRC_FLAG_BLUR) ? 1 : 0, nullptr, half ? 1 : 0};
    const int np = build_rgb_backward_phases(w, b, ph, kMaxPhases,
                                             (flags & HRC_FLAG_REUSE_PYRAMID) == 0);
    return run_phases(ph, np, s);
}

// ---- several diffuse bounces ------------------------------------------------

static constexpr int kMaxBounces = 64;

// Workspace of the bounce loop: one solve's workspace, then the source buffer,
// and for the reverse dLoss/dF of the previous bounce, dLoss/d eps and
// dLoss/d sigma of one bounce, and the fluence of bounces 0..K-2.
struct BounceLayout {
    Layout solve;
    size_t src = 0, g = 0, dE = 0, dS = 0, saved = 0, field = 0, total = 0;
};

static BounceLayout bounce_layout(int N, int bounces, bool backward, int group) {
    BounceLayout M;
    M.solve = make_layout(N, backward, group);
    M.field = align256((size_t(1) << (2 * N)) * sizeof(float));
    size_t off = align256(M.solve.total);
    M.src = off;
    off += M.field;
    if (backward) {
        M.g = off;
        off += M.field;
        M.dE = off;
        off += M.field;
        M.dS = off;
        off += M.field;
        M.saved = off;
        off += (size_t)(bounces - 1) * M.field;
    }
    M.total = off;
    return M;
}

static int phase_level(const Phase &p) {
    switch (p.kind) {
        case PH_UP: return p.a.up.n;
        case PH_DOWN: return p.a.down.n;
        case PH_DOWN_ADJ: return p.a.da.n;
        case PH_DT: return p.a.dt.n;
        default: return -1;
    }
}

hrc_status hrc_multibounce_workspace_bytes(int log2_size, int bounces, unsigned flags,
                                           size_t *forward_bytes, size_t *backward_bytes) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (bounces < 1 || bounces > kMaxBounces) return HRC_ERR_INVALID_ARG;
    if (flags & ~(HRC_FLAG_VALIDATE | HRC_FLAG_QUADRANTS_MASK)) return HRC_ERR_UNSUPPORTED;
    if (forward_bytes)
        *forward_bytes =
            bounce_layout(log2_size, bounces, false, forward_group(log2_size, flags)).total;
    if (backward_bytes) *backward_bytes = bounce_layout(log2_size, bounces, true, 4).total;
    return HRC_OK;
}

hrc_status hrc_multibounce_forward(hrc_context *ctx, int log2_size, const float *emission,
                                   const float *sigma_t, const float *albedo, int bounces,
                                   float *fluence, void *workspace, size_t workspace_bytes,
                                   void *stream, unsigned flags) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (!aligned16(emission) || !aligned16(sigma_t) || !aligned16(albedo) ||
        !aligned16(fluence) || !aligned16(workspace) || bounces < 1 || bounces > kMaxBounces)
        return HRC_ERR_INVALID_ARG;
    if (flags & ~(HRC_FLAG_VALIDATE | HRC_FLAG_QUADRANTS_MASK)) return HRC_ERR_UNSUPPORTED;
    const BounceLayout M =
        bounce_layout(log2_size, bounces, false, forward_group(log2_size, flags));
    if (workspace_bytes < M.total) return HRC_ERR_WORKSPACE;
    if (!ctx) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(workspace);
    Ws w{base, M.solve};
    if (flags & HRC_FLAG_VALIDATE) {
        st = validate_inputs(w, emission, sigma_t, s);
        if (st == HRC_OK) st = validate_inputs(w, albedo, albedo, s);
        if (st != HRC_OK) return st;
    }
    const size_t SS = M.solve.S * M.solve.S;
    float *src = reinterpret_cast<float *>(base + M.src);
    const float *env = ctx->has_env ? ctx->env : nullptr;
    Phase ph[kMaxPhases];
    for (int k = 0; k < bounces; ++k) {
        // bounce k: source eps_0 (k = 0) or eps_0 + a sigma F_{k-1} / (2 pi)
        if (k > 0 &&
            launch_scatter_source(emission, sigma_t, albedo, fluence, src, SS, s) != hipSuccess)
            return HRC_ERR_HIP;
        SolveBuffers b{k == 0 ? emission : src, sigma_t, fluence, nullptr, nullptr, nullptr,
                       0, env};
        const int np = build_solve_phases(w, b, false, nullptr, ph, kMaxPhases);
        st = run_phases(ph, np, s);
        if (st != HRC_OK) return st;
    }
    return HRC_OK;
}

hrc_status hrc_multibounce_backward(hrc_context *ctx, int log2_size, const float *emission,
                                    const float *sigma_t, const float *albedo, int bounces,
                                    const float *grad_fluence, float *grad_emission,
                                    float *grad_sigma_t, float *grad_albedo, void *workspace,
                                    size_t workspace_bytes, void *stream, unsigned flags) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    if (!aligned16(emission) || !aligned16(sigma_t) || !aligned16(albedo) ||
        !aligned16(grad_fluence) || !aligned16(grad_emission) || !aligned16(grad_sigma_t) ||
        !aligned16(grad_albedo) || !aligned16(workspace) || bounces < 1 ||
        bounces > kMaxBounces)
        return HRC_ERR_INVALID_ARG;
    if (flags & ~(HRC_FLAG_VALIDATE | HRC_FLAG_QUADRANTS_MASK)) return HRC_ERR_UNSUPPORTED;
    const BounceLayout M = bounce_layout(log2_size, bounces, true, 4);
    if (workspace_bytes < M.total) return HRC_ERR_WORKSPACE;
    if (!ctx) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(workspace);
    Ws w{base, M.solve};
    if (flags & HRC_FLAG_VALIDATE) {
        st = validate_inputs(w, emission, sigma_t, s);
        if (st == HRC_OK) st = validate_inputs(w, albedo, albedo, s);
        if (st != HRC_OK) return st;
    }
    const size_t SS = M.solve.S * M.solve.S;
    float *src = reinterpret_cast<float *>(base + M.src);
    float *gbuf = reinterpret_cast<float *>(base + M.g);
    float *dE = reinterpret_cast<float *>(base + M.dE);
    float *dS = reinterpret_cast<float *>(base + M.dS);
    auto saved = [&](int k) { return reinterpret_cast<float *>(base + M.saved + k * M.field); };
    const float *env = ctx->has_env ? ctx->env : nullptr;
    Phase ph[kMaxPhases];
    // the sources of bounces 1..K-1 need F_0..F_{K-2}: recompute and keep them
    // (every cascade level kept, so the solve fits the reverse's workspace)
    for (int k = 0; k + 1 < bounces; ++k) {
        if (k > 0 && launch_scatter_source(emission, sigma_t, albedo, saved(k - 1), src, SS,
                                           s) != hipSuccess)
            return HRC_ERR_HIP;
        SolveBuffers b{k == 0 ? emission : src, sigma_t, saved(k), nullptr, nullptr, nullptr,
                       0, env};
        const int np = build_solve_phases(w, b, true, nullptr, ph, kMaxPhases);
        st = run_phases(ph, np, s);
        if (st != HRC_OK) return st;
    }
    // reverse: bounce K-1 first; each bounce's dLoss/d eps feeds the previous
    // bounce's dLoss/dF through the source
    const float *gin = grad_fluence;
    for (int k = bounces - 1; k >= 0; --k) {
        if (k > 0 && launch_scatter_source(emission, sigma_t, albedo, saved(k - 1), src, SS,
                                           s) != hipSuccess)
            return HRC_ERR_HIP;
        SolveBuffers b{k == 0 ? emission : src, sigma_t, nullptr, gin, dE, dS, 0, env};
        const int np = build_solve_phases(w, b, true, nullptr, ph, kMaxPhases);
        st = run_phases(ph, np, s);
        if (st != HRC_OK) return st;
        if (launch_scatter_adj(dE, dS, k > 0 ? saved(k - 1) : nullptr, sigma_t, albedo, gbuf,
                               grad_emission, grad_sigma_t, grad_albedo, SS,
                               k == bounces - 1 ? 1 : 0, s) != hipSuccess)
            return HRC_ERR_HIP;
        gin = gbuf;
    }
    return HRC_OK;
}

hrc_status hrc_profile_solve(hrc_context *ctx, int log2_size, const float *emission,
                             const float *sigma_t, float *fluence, const float *grad_fluence,
                             float *grad_emission, float *grad_sigma_t, void *workspace,
                             size_t workspace_bytes, void *stream, float *pass_ms,
                             int *pass_kind, int *pass_level, int max_passes, int *count) {
    hrc_status st = check_shape(log2_size);
    if (st != HRC_OK) return st;
    const bool bwd = grad_fluence != nullptr;
    if (!aligned16(emission) || !aligned16(sigma_t) || !aligned16(workspace))
        return HRC_ERR_INVALID_ARG;
    if (bwd ? (!aligned16(grad_emission) || !aligned16(grad_sigma_t)) : !aligned16(fluence))
        return HRC_ERR_INVALID_ARG;
    if (!pass_ms || !pass_kind || !pass_level || !count || max_passes < 0)
        return HRC_ERR_INVALID_ARG;
    Layout L = bwd ? make_layout(log2_size, true)
                   : make_layout(log2_size, false, forward_group(log2_size, 0));
    if (workspace_bytes < L.total) return HRC_ERR_WORKSPACE;
    if (!ctx) return HRC_ERR_INVALID_ARG;
    DeviceGuard g(ctx->device);
    if (!g.ok) return HRC_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ws w{static_cast<char *>(workspace), L};
    Phase ph[kMaxPhases];
    const float *env = ctx->has_env ? ctx->env : nullptr;
    SolveBuffers b = bwd ? SolveBuffers{emission, sigma_t, nullptr, grad_fluence, grad_emission,
                                        grad_sigma_t, 0, env}
                         : SolveBuffers{emission, sigma_t, fluence, nullptr, nullptr, nullptr,
                                        0, env};
    const int np = build_solve_phases(w, b, bwd, nullptr, ph, kMaxPhases);
    // events 2i, 2i+1: start and end of pass i, recorded by the launch itself
    std::vector<hipEvent_t> ev(2 * np, nullptr);
    st = HRC_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) st = HRC_ERR_HIP;
    for (int i = 0; i < np && st == HRC_OK; ++i) {
        if (launch_phase(ph[i], s, ev[2 * i], ev[2 * i + 1]) != hipSuccess) st = HRC_ERR_HIP;
    }
    if (st == HRC_OK && np > 0 && hipEventSynchronize(ev[2 * np - 1]) != hipSuccess)
        st = HRC_ERR_HIP;
    for (int i = 0; i < np && st == HRC_OK; ++i) {
        if (i >= max_passes) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess) st = HRC_ERR_HIP;
        pass_ms[i] = ms;
        pass_kind[i] = ph[i].kind;
        pass_level[i] = phase_level(ph[i]);
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    *count = np;
    return st;
}

}  // extern "C"
