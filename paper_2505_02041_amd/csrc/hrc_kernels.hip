// HIP kernels (gfx950) of Holographic Radiance Cascades: forward and adjoint.
//
// Frames.  Each quadrant solve works in a frame (u, w) whose +u axis faces the
// quadrant (Section 4: the solve for [-pi/4, pi/4] is rotated four times,
// Algorithm 1, Lighting).  Quadrant q reads the scene as
//   q = 0 (+x): E[u][w] = img[w][u]
//   q = 1 (-x): E[u][w] = img[w][S-1-u]
//   q = 2 (+y): E[u][w] = img[u][w]
//   q = 3 (-y): E[u][w] = img[S-1-u][w]
// Each solve is mirror symmetric in w, so flips stand in for rotations.  The
// passes that read the image (traced levels, tail, their adjoints) stage an
// image tile in LDS and address it in each quadrant's frame.
//
// Storage (per quadrant, y = w fastest so that 64 lanes read 64 consecutive y):
//   T_n  float2 (L, T)  [S >> n][2^n + 1][S]   index (x*(2^n+1) + k)*S + y
//   R_n  float          [S >> n][2^n][S]       index ((x << n) | ii)*S + y
// (T_n as a pair of IEEE halves instead, same index, in the forward with the
// 16-bit storage of Section 5.)
// Probe (n, x, y) sits at the centre of pixel (x*2^n, y).  Outside the grid
// there is no light unless an environment map is set: an interval starting
// off-grid is <0, 1>, an angular fluence off-grid is 0 (or the map's), and
// R_N = 0 (Section 4.2).
//
// Every pass is in gather form: each output element has one writer, which
// reads what it needs, so results do not depend on the launch shape and need
// no atomics.
#include <hip/hip_ext.h>

#include "hrc_internal.h"

namespace hrc {

// A_m(jj) of Eq. 13 for m = 0..12 at offset 2^m - 1 (uploaded by the host).
__constant__ float c_cone[kConeTable];

// Half lengths of the traced rays' pieces (below): every traced chord through
// a pixel is one or two of these.
constexpr float kH2 = 0.70710678118654752f;  // sqrt(2)/2
constexpr float kQ5 = 0.55901699437494742f;  // sqrt(5)/4

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Work-tile id for block b of nb: consecutive tiles land on the same XCD (the
// hardware deals blocks round-robin over 8 XCDs), so neighbouring rows that
// share input rows, and neighbouring image tiles that share a halo, share an
// L2 (it cut the traced levels' and the tail's HBM reads of their halos).
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
    unsigned xcd = b & 7u, local = b >> 3;
    unsigned q = nb >> 3, r = nb & 7u;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// The same with the tiles dealt to the XCDs in blocks of 2^lb, round robin
// (the last partial round split as above), so that the XCDs work on nearby
// addresses at any time instead of addresses an eighth of the pass apart.
__device__ __forceinline__ unsigned xcd_tile_blk(unsigned b, unsigned nb, unsigned lb) {
    if (lb == 0) return xcd_tile(b, nb);
    const unsigned xcd = b & 7u, local = b >> 3;
    const unsigned full = nb >> (3 + lb);
    if (local < (full << lb))
        return ((((local >> lb) << 3) + xcd) << lb) + (local & ((1u << lb) - 1));
    const unsigned rem = nb - (full << (3 + lb));
    return (full << (3 + lb)) + xcd_tile(xcd + 8u * (local - (full << lb)), rem);
}

// <L, T> of a chord of length ell through a uniform pixel (Eq. 2-4):
// T = exp(-tau), L = eps*ell*(1 - exp(-tau))/tau, tau = sig*ell.
//
// exp(-tau) is the hardware base-2 exponential of -tau*log2(e): its relative
// error grows as tau * 2^-24, about 2e-6 at tau = 25, where T is 1e-11.
// phi(tau) = (1 - exp(-tau)) / tau is its Taylor polynomial through tau^5
// below 1/8 (truncation under 1e-9, where the difference would cancel) and
// the difference times the hardware reciprocal above.
__device__ __forceinline__ float exp_neg(float tau) {
    return __builtin_amdgcn_exp2f(tau * -1.44269504088896341f);
}

__device__ __forceinline__ float cell_phi(float tau) {
    const float p =
        1.0f - tau * (0.5f - tau * (1.0f / 6.0f - tau * (1.0f / 24.0f -
                                                         tau * (1.0f / 120.0f - tau * (1.0f / 720.0f)))));
    const float d = (1.0f - exp_neg(tau)) * __builtin_amdgcn_rcpf(tau);
    return tau < 0.125f ? p : d;
}

__device__ __forceinline__ float2 cell_interval(float e, float s, float ell) {
    float tau = s * ell;
    return make_float2(e * ell * cell_phi(tau), exp_neg(tau));
}

// Eq. 7: near interval first.
__device__ __forceinline__ float2 merge(float2 n, float2 f) {
    return make_float2(fmaf(n.y, f.x, n.x), n.y * f.y);
}

// Three radiance channels over one medium (RGB): (L_r, L_g, L_b, T), each
// channel merged exactly as the one-channel interval.
__device__ __forceinline__ float4 merge(float4 n, float4 f) {
    return make_float4(fmaf(n.w, f.x, n.x), fmaf(n.w, f.y, n.y), fmaf(n.w, f.z, n.z), n.w * f.w);
}

// The RGB pixel interval: the one-channel expression per channel, with the
// attenuation's phi and exp(-tau) shared.
__device__ __forceinline__ float4 cell_interval_rgb(float e0, float e1, float e2, float s,
                                                    float ell) {
    const float tau = s * ell;
    const float phi = cell_phi(tau);
    return make_float4(e0 * ell * phi, e1 * ell * phi, e2 * ell * phi, exp_neg(tau));
}

__device__ __forceinline__ int frame_row(int q, int u, int S) {
    return (q & 1) ? S - 1 - u : u;
}

// The environment's angular fluence in cone jj of level m (0 without one):
// what an angular fluence looked up outside the grid reads, and R_N.
__device__ __forceinline__ float env_fluence(const float *envq, int m, int jj) {
    return envq ? envq[(1 << m) - 1 + jj] : 0.f;
}

// ---------------------------------------------------------------------------
// Phase bodies.  Each computes one work tile; a standalone kernel runs one tile
// per block and the persistent batch kernel runs tiles pulled from its queue,
// so both paths execute the same code.  Elementwise phases cover 256*U
// consecutive output elements per tile (U elements per thread, 256 apart).
// ---------------------------------------------------------------------------

// Two consecutive y per thread: y is even and every shift is even (except
// the odd-column shifts 2e - 1 of merge-down level 0, read element-wise), so a
// pair of intervals is one aligned 16-byte load and a pair of angular
// fluences one aligned 8-byte load, and both members of a shifted pair are in
// or out of the grid together.
__device__ __forceinline__ float4 ld_pair(const float2 *p) {
    return *reinterpret_cast<const float4 *>(p);
}
__device__ __forceinline__ float2 lo(float4 v) { return make_float2(v.x, v.y); }
__device__ __forceinline__ float2 hi(float4 v) { return make_float2(v.z, v.w); }
__device__ __forceinline__ float4 pair(float2 a, float2 b) { return make_float4(a.x, a.y, b.x, b.y); }
__device__ __forceinline__ void st_pair(float2 *p, float4 v) { *reinterpret_cast<float4 *>(p) = v; }
__device__ __forceinline__ void st_iv(float2 *p, float2 v) { *p = v; }
__device__ __forceinline__ void st_iv(float4 *p, float4 v) { *p = v; }
template <typename I> __device__ __forceinline__ I empty_interval();
template <> __device__ __forceinline__ float2 empty_interval<float2>() { return make_float2(0.f, 1.f); }
template <> __device__ __forceinline__ float4 empty_interval<float4>() {
    return make_float4(0.f, 0.f, 0.f, 1.f);
}

// The 16-bit interval storage of Section 5 (HRC_FLAG_HALF_INTERVALS, forward
// only): an interval is a pair of IEEE half floats (L, T), computed in FP32 and
// rounded to nearest even once when it is stored; a pair of intervals is one
// 8-byte load.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

// An FP32 value rounded to half.  The value is first pinned in a register, so
// that the compiler cannot fuse the arithmetic that produced it with the
// narrowing (a mixed-precision FMA that rounds the exact result to half once,
// e.g. v_fma_mixlo_f16): the stored half is always the FP32 result rounded to
// nearest even, whatever the code around it.
__device__ __forceinline__ _Float16 to_half(float v) {
    asm volatile("" : "+v"(v));
    return (_Float16)v;
}
// A loaded operand pinned in a register at the point where every load of a
// pass has been issued.  Loads under conditions uniform over the wave would
// otherwise draw the arithmetic that uses them into each conditional block,
// and each block would then wait for its own loads: the pins keep the loads
// of all the blocks in flight together, so the wave waits for memory once.
__device__ __forceinline__ void pin(float &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(float2 &v) { pin(v.x); pin(v.y); }
__device__ __forceinline__ void pin(float4 &v) { pin(v.x); pin(v.y); pin(v.z); pin(v.w); }

__device__ __forceinline__ float4 ld_pair(const half2_t *p) {
    const half4_t v = *reinterpret_cast<const half4_t *>(p);
    return make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
}
__device__ __forceinline__ void st_pair(half2_t *p, float4 v) {
    half4_t h;
    h.x = to_half(v.x);
    h.y = to_half(v.y);
    h.z = to_half(v.z);
    h.w = to_half(v.w);
    *reinterpret_cast<half4_t *>(p) = h;
}
__device__ __forceinline__ void st_iv(half2_t *p, float2 v) {
    half2_t h;
    h.x = to_half(v.x);
    h.y = to_half(v.y);
    *p = h;
}

// The transmittance of one stored interval, FP32 or 16-bit.
__device__ __forceinline__ float iv_t(const float2 *p) { return p->y; }
__device__ __forceinline__ float iv_t(const half2_t *p) { return (float)(*p).y; }

template <typename TS>
__device__ __forceinline__ float4 far_pair(const TS *row, int yf, int S) {
    return (yf >= 0 && yf < S) ? ld_pair(row + yf) : make_float4(0.f, 1.f, 0.f, 1.f);
}

// Four consecutive 16-bit intervals (two pairs) at y, y a multiple of 4, as
// one 16-byte load, and their conversion to two FP32 pairs.
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ void cvt_quad(half8_t v, float4 &a, float4 &b) {
    a = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    b = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
}
// Raw 16-bit loads pinned as they are, before their conversion (see pin).
__device__ __forceinline__ void pin(half8_t &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(half4_t &v) { asm volatile("" : "+v"(v)); }
// A far row's two interval pairs at yf and yf + 2 (yf even) as raw halves,
// outside [0, S) from a clamped address, with the flags that select <0, 1>
// for them once converted.
__device__ __forceinline__ void far_pairs_raw(const half2_t *row, int yf, int S, half4_t h[2],
                                              bool in[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        in[j] = (unsigned)(yf + 2 * j) < (unsigned)S;
        h[j] = *reinterpret_cast<const half4_t *>(row + (in[j] ? yf + 2 * j : 0));
    }
}
// An interval pair as stored (FP32, or four halves), loaded without its
// conversion, so that it can be pinned before it is used.
template <typename TS> struct PairRaw;
template <> struct PairRaw<float2> { using type = float4; };
template <> struct PairRaw<half2_t> { using type = half4_t; };
template <typename TS> __device__ __forceinline__ typename PairRaw<TS>::type raw_zero() {
    return typename PairRaw<TS>::type{0, 0, 0, 0};
}
__device__ __forceinline__ float4 ld_pair_raw(const float2 *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ half4_t ld_pair_raw(const half2_t *p) { return *reinterpret_cast<const half4_t *>(p); }
__device__ __forceinline__ float4 cvt_pair(float4 v) { return v; }
__device__ __forceinline__ float4 cvt_pair(half4_t v) {
    return make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
}
__device__ __forceinline__ float4 far_pair_cvt(half4_t v, bool in) {
    return in ? make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w)
              : make_float4(0.f, 1.f, 0.f, 1.f);
}
__device__ __forceinline__ void st_quad(half2_t *p, float4 a, float4 b) {
    half8_t h;
    h[0] = to_half(a.x); h[1] = to_half(a.y); h[2] = to_half(a.z); h[3] = to_half(a.w);
    h[4] = to_half(b.x); h[5] = to_half(b.y); h[6] = to_half(b.z); h[7] = to_half(b.w);
    *reinterpret_cast<half8_t *>(p) = h;
}
__device__ __forceinline__ void st_quad(float2 *, float4, float4) {}  // not used with FP32

// One RGB interval (L_r, L_g, L_b, T): FP32, or four IEEE halves (the 16-bit
// storage, rounded to nearest even once when stored).
__device__ __forceinline__ float4 ld4(const float4 *p) { return *p; }
__device__ __forceinline__ float4 ld4(const half4_t *p) {
    const half4_t v = *p;
    return make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
}
__device__ __forceinline__ void st_iv(half4_t *p, float4 v) {
    half4_t h;
    h.x = to_half(v.x);
    h.y = to_half(v.y);
    h.z = to_half(v.z);
    h.w = to_half(v.w);
    *p = h;
}

// Traced levels T_0, T_1, T_2 (Algorithm 1, first loop), for all four
// quadrants from one 32x32 image tile (T_2 alone when the forward's tail folds
// the intervals of T_0 and T_1 itself).
//
// A chord of length 2a through a uniform pixel is the merge of two chords of
// length a through it (Eq. 5-6), and every chord of the traced rays is either
// 1/2 or 1 (axis rays), sqrt(2)/2 or sqrt(2) (diagonals), sqrt(5)/4 or
// sqrt(5)/2 (slope 1/2).  So each pixel needs only three intervals, for the
// half lengths 1/2, sqrt(2)/2 and sqrt(5)/4, and every traced ray is a fold of
// 2^(n+1) half pieces.  The block computes the three intervals of its tile
// plus a 4-pixel halo once into LDS (out-of-grid pixels are vacuum <0, 1>)
// and then folds the 4 x 4864 rays whose probes lie in the tile, each thread
// every direction of one probe at a time.
// Thread index within a 256-thread work tile.  Every pass body is written for
// 256 threads and takes this index as its `tid` argument; the persistent
// kernel runs several tiles side by side in one block, one per 256-thread
// quarter, and passes each body an opaque copy (see run_phase).
__device__ __forceinline__ int ltid() { return (int)(threadIdx.x & 255u); }

constexpr int kSeedHalo = 4;
template <int TILE> struct SeedTile {
    static constexpr int span = TILE + 2 * kSeedHalo;  // tile plus halo
    static constexpr int pitch = span + 1;            // padded LDS row pitch
    static constexpr int lds = 3 * span * pitch * 8;  // three intervals per pixel
};

// Half pieces of the traced rays: (du, dw) from the probe's pixel and the
// half-length id (0: 1/2, 1: sqrt(2)/2, 2: sqrt(5)/4), in order from the probe.
// Stencil id: n = 0 -> k, n = 1 -> 2 + k, n = 2 -> 5 + k; 2^(n+1) pieces each.
constexpr signed char kHpDu[10][8] = {
    {0, 1}, {0, 1},
    {0, 1, 1, 2}, {0, 1, 1, 2}, {0, 1, 1, 2},
    {0, 1, 1, 2, 2, 3, 3, 4}, {0, 1, 1, 2, 2, 3, 3, 4}, {0, 1, 1, 2, 2, 3, 3, 4},
    {0, 1, 1, 2, 2, 3, 3, 4}, {0, 1, 1, 2, 2, 3, 3, 4}};
constexpr signed char kHpDw[10][8] = {
    {0, -1}, {0, 1},
    {0, -1, -1, -2}, {0, 0, 0, 0}, {0, 1, 1, 2},
    {0, -1, -1, -2, -2, -3, -3, -4}, {0, 0, -1, -1, -1, -1, -2, -2},
    {0, 0, 0, 0, 0, 0, 0, 0}, {0, 0, 1, 1, 1, 1, 2, 2}, {0, 1, 1, 2, 2, 3, 3, 4}};
constexpr unsigned char kHpLen[10][8] = {
    {1, 1}, {1, 1},
    {1, 1, 1, 1}, {0, 0, 0, 0}, {1, 1, 1, 1},
    {1, 1, 1, 1, 1, 1, 1, 1}, {2, 2, 2, 2, 2, 2, 2, 2}, {0, 0, 0, 0, 0, 0, 0, 0},
    {2, 2, 2, 2, 2, 2, 2, 2}, {1, 1, 1, 1, 1, 1, 1, 1}};

// Rays of traced level n of quadrant q whose probes lie in the tile.  A
// thread owns one probe (column xl, row w) at a time and folds all its
// directions (unrolled: the piece offsets are uniform over the wave), so the
// LDS base and the output address are computed once per probe; lanes run
// along w, so each direction's stores are contiguous rows.
template <int TILE, int n, typename TS, typename I = float2>
__device__ __forceinline__ void seed_level_rays(const I *iv, const SeedArgs &a, int q,
                                                int slot, int r0, int c0, int tid) {
    using G = SeedTile<TILE>;
    constexpr int dirs = (1 << n) + 1, cols = TILE >> n, pieces = 2 << n;
    constexpr int per_pass = 256 / TILE;  // probe columns per pass of the block
    const int S = 1 << a.N;
    TS *out = reinterpret_cast<TS *>(n == 0 ? a.T0 : n == 1 ? a.T1 : a.T2);
    const size_t qoff = n == 0 ? a.e0 : n == 1 ? a.e1 : a.e2;
    // frame of quadrant q: +x (u, w) = (c, r); -x (S-1-c, r); +y (r, c); -y (S-1-r, c)
    const int u_lo = q == 0 ? c0 : q == 1 ? S - TILE - c0 : q == 2 ? r0 : S - TILE - r0;
    const int w_lo = q < 2 ? r0 : c0;
    const int su = q == 0 ? 1 : q == 1 ? -1 : q == 2 ? G::pitch : -G::pitch;
    const int sw = q < 2 ? G::pitch : 1;
    const int wl = tid % TILE;
    const int w = w_lo + wl;
    constexpr int sid0 = n == 0 ? 0 : n == 1 ? 2 : 5;
    for (int xl = tid / TILE; xl < cols; xl += per_pass) {
        const int u = u_lo + (xl << n);
        if (u < 0 || u >= S || w >= S) continue;
        int lr, lc;
        if (q < 2) { lr = w - r0; lc = (q == 0 ? u : S - 1 - u) - c0; }
        else { lc = w - c0; lr = (q == 2 ? u : S - 1 - u) - r0; }
        const I *ivp = iv + (lr + kSeedHalo) * G::pitch + lc + kSeedHalo;
        TS *o = out + slot * qoff + (size_t)(u >> n) * dirs * S + w;
#pragma unroll
        for (int k = 0; k < dirs; ++k) {
            I acc = empty_interval<I>();
#pragma unroll
            for (int j = 0; j < pieces; ++j) {
                const int off = kHpLen[sid0 + k][j] * (G::span * G::pitch) +
                                kHpDu[sid0 + k][j] * su + kHpDw[sid0 + k][j] * sw;
                acc = merge(acc, ivp[off]);
            }
            st_iv(o + (size_t)k * S, acc);
        }
    }
}

// TILE x TILE image pixels per work tile (32 for the standalone kernel, 16
// inside the persistent kernel, whose one LDS buffer serves every pass); the
// per-ray arithmetic is the same for both.
template <int TILE, typename TS>
__device__ void body_seed(const SeedArgs &a, unsigned tile, char *lds, int tid) {
    using G = SeedTile<TILE>;
    float2 *iv = reinterpret_cast<float2 *>(lds);
    const int S = 1 << a.N;
    const int tiles = (S + TILE - 1) / TILE;
    const int r0 = (int)(tile / tiles) * TILE, c0 = (int)(tile % tiles) * TILE;
    // the fields of the tile and its halo: every load of the thread first
    // (cells outside the grid from a clamped address, then 0), then the
    // intervals, so the block waits for memory once
    constexpr int cells = G::span * G::span, NI = (cells + 255) / 256;
    float ev[NI], gv[NI];
    bool inside[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = tid + 256 * it;
        const int lr = i / G::span, lc = i % G::span;
        const int r = r0 - kSeedHalo + lr, c = c0 - kSeedHalo + lc;
        inside[it] = i < cells && (unsigned)r < (unsigned)S && (unsigned)c < (unsigned)S;
        const unsigned o = inside[it] ? (unsigned)(r * S + c) : 0u;
        ev[it] = a.eps[o];
        gv[it] = a.sig[o];
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        pin(ev[it]);
        pin(gv[it]);
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = tid + 256 * it;
        if (i < cells) {
            const float e = inside[it] ? ev[it] : 0.f, g = inside[it] ? gv[it] : 0.f;
            const int l = (i / G::span) * G::pitch + i % G::span;
            iv[l] = cell_interval(e, g, 0.5f);
            iv[G::span * G::pitch + l] = cell_interval(e, g, kH2);
            iv[2 * G::span * G::pitch + l] = cell_interval(e, g, kQ5);
        }
    }
    __syncthreads();
    for (int g = 0; g < a.nq; ++g) {
        if (a.first <= 0) seed_level_rays<TILE, 0, TS>(iv, a, a.q0 + g, g, r0, c0, tid);
        if (a.first <= 1) seed_level_rays<TILE, 1, TS>(iv, a, a.q0 + g, g, r0, c0, tid);
        seed_level_rays<TILE, 2, TS>(iv, a, a.q0 + g, g, r0, c0, tid);
    }
    __syncthreads();
}

// Pairs of consecutive y per thread in the merges: one with FP32 intervals
// (a pair is a 16-byte load), two with 16-bit ones (so that a thread still
// has 16 bytes of each row in flight).
template <typename TS> constexpr int merge_pairs() { return sizeof(TS) == 4 ? 2 : 1; }

// floor(r / d) for a row index r = x d + k of a level (d = 2^n + 1 directions,
// 0 <= k < d, x below 2^12, so r below 2^14): the single-precision estimate
// is within one of x, and one correction each way makes it exact, in a few
// instructions where an integer division takes some thirty.
__device__ __forceinline__ unsigned div_rows(unsigned r, unsigned d) {
    unsigned x = (unsigned)((float)r * __builtin_amdgcn_rcpf((float)d));
    x = x * d > r ? x - 1 : x;
    x = (x + 1) * d <= r ? x + 1 : x;
    return x;
}

// Merge up: T_n from T_{n-1} (Section 4.1, Eq. 18-20), for n < N.  The top
// level is never stored: the merge down reads T_N only through the even
// directions of its one column (the doubled edges of Eq. 15-17), and builds
// those itself from T_{N-1}.
template <typename TS>
__device__ void body_merge_up(const UpArgs &a, unsigned tile, int U, int tid) {
    constexpr int P = merge_pairs<TS>();
    const int N = a.N, S = 1 << N, n = a.n;
    const int h = 1 << (n - 1);
    const int dirs = 2 * h + 1, pdirs = h + 1;
    const unsigned rpq = (unsigned)(S >> n) * dirs;
    const size_t total = (size_t)a.nq * rpq * (S / (2 * P));
    for (int uu = 0; uu < U; ++uu) {
        const size_t idx = ((size_t)tile * U + uu) * 256 + tid;
        if (idx >= total) return;
        const int y0 = (int)(idx & (S / (2 * P) - 1)) * 2 * P;
        const unsigned row = (unsigned)(idx >> (N - (P == 2 ? 2 : 1)));
        const int q = (row >= rpq) + (row >= 2 * rpq) + (row >= 3 * rpq);
        const unsigned rk = row - (unsigned)q * rpq;
        const int x = (int)div_rows(rk, (unsigned)dirs), k = (int)(rk - (unsigned)x * dirs);
        const unsigned r = rk;  // output row (x, k)
        // 32-bit element offsets (a level of four quadrants holds fewer than
        // 2^28 entries)
        const TS *near = reinterpret_cast<const TS *>(a.Tp) +
                         ((unsigned)q * (unsigned)a.ep + ((unsigned)(2 * x) * pdirs << N));
        const TS *far = near + ((unsigned)pdirs << N);
        float4 res[P];
        if constexpr (P == 2) {
            // 16-bit intervals: each near row read as one quad (two pairs) per
            // thread, each far row as two pairs (its shift is only even); the
            // raw halves are all loaded, and pinned, before any is converted
            if ((k & 1) == 0) {
                const int kk = k >> 1;
                half8_t hn = *reinterpret_cast<const half8_t *>(near + (size_t)kk * S + y0);
                half4_t hf[2];
                bool in[2];
                far_pairs_raw(far + (size_t)kk * S, y0 + 2 * kk - h, S, hf, in);
                pin(hn);
                pin(hf[0]);
                pin(hf[1]);
                float4 nv[2];
                cvt_quad(hn, nv[0], nv[1]);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const float4 fv = far_pair_cvt(hf[j], in[j]);
                    res[j] = pair(merge(lo(nv[j]), lo(fv)), merge(hi(nv[j]), hi(fv)));
                }
            } else {
                const int ka = (k + 1) >> 1, kb = (k - 1) >> 1;
                half8_t hna = *reinterpret_cast<const half8_t *>(near + (size_t)ka * S + y0);
                half8_t hnb = *reinterpret_cast<const half8_t *>(near + (size_t)kb * S + y0);
                half4_t hfa[2], hfb[2];
                bool ina[2], inb[2];
                far_pairs_raw(far + (size_t)kb * S, y0 + 2 * ka - h, S, hfa, ina);
                far_pairs_raw(far + (size_t)ka * S, y0 + 2 * kb - h, S, hfb, inb);
                pin(hna);
                pin(hnb);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    pin(hfa[j]);
                    pin(hfb[j]);
                }
                float4 na[2], nb[2];
                cvt_quad(hna, na[0], na[1]);
                cvt_quad(hnb, nb[0], nb[1]);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const float4 fa = far_pair_cvt(hfa[j], ina[j]), fb = far_pair_cvt(hfb[j], inb[j]);
                    const float2 p0 = merge(lo(na[j]), lo(fa)), m0 = merge(lo(nb[j]), lo(fb));
                    const float2 p1 = merge(hi(na[j]), hi(fa)), m1 = merge(hi(nb[j]), hi(fb));
                    res[j] = make_float4(0.5f * (p0.x + m0.x), 0.5f * (p0.y + m0.y),
                                         0.5f * (p1.x + m1.x), 0.5f * (p1.y + m1.y));
                }
            }
        } else {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int y = y0 + 2 * j;
            if ((k & 1) == 0) {
                // Eq. 18: p -> p + v_{n-1}(k/2) -> p + v_n(k), exact.
                const int kk = k >> 1;
                const float4 nv = ld_pair(near + (size_t)kk * S + y);
                const float4 fv = far_pair(far + (size_t)kk * S, y + 2 * kk - h, S);
                res[j] = pair(merge(lo(nv), lo(fv)), merge(hi(nv), hi(fv)));
            } else {
                // Eq. 19-20: mean of the two bent paths through directions (k+-1)/2.
                const int ka = (k + 1) >> 1, kb = (k - 1) >> 1;
                const float4 na = ld_pair(near + (size_t)ka * S + y);
                const float4 nb = ld_pair(near + (size_t)kb * S + y);
                const float4 fa = far_pair(far + (size_t)kb * S, y + 2 * ka - h, S);
                const float4 fb = far_pair(far + (size_t)ka * S, y + 2 * kb - h, S);
                const float2 p0 = merge(lo(na), lo(fa)), m0 = merge(lo(nb), lo(fb));
                const float2 p1 = merge(hi(na), hi(fa)), m1 = merge(hi(nb), hi(fb));
                res[j] = make_float4(0.5f * (p0.x + m0.x), 0.5f * (p0.y + m0.y),
                                     0.5f * (p1.x + m1.x), 0.5f * (p1.y + m1.y));
            }
        }
        }
        TS *out = reinterpret_cast<TS *>(a.T) + ((unsigned)q * (unsigned)a.e + (r << N) + (unsigned)y0);
        if constexpr (P == 2) {
            st_quad(out, res[0], res[1]);
        } else {
            st_pair(out, res[0]);
        }
    }
}

template <typename TS>
__device__ __forceinline__ float4 far_pair_sel(const TS *row, int yf, int S) {
    const bool in = (unsigned)yf < (unsigned)S;
    const float4 v = ld_pair(row + (in ? yf : 0));
    return in ? v : make_float4(0.f, 1.f, 0.f, 1.f);
}

// R_{n+1} pair at (c, jj) and rows (y, y+1), y even, of the quadrant whose
// level starts at element rq, or the environment's fluence e outside the grid
// (column c past the last, or y outside [0, S)): a clamped address and a
// select.  Element offsets are 32-bit: a level of four quadrants holds at
// most 2^26 entries (S <= 4096), three channel planes of it 3 x 2^26.
__device__ __forceinline__ float2 r_pair_sel(const float *R, unsigned rq, int N, int m, int c,
                                             int jj, int y, float e) {
    const int S = 1 << N;
    const bool in = c < (S >> m) && (unsigned)y < (unsigned)S;
    const unsigned at = rq + ((unsigned)(((in ? c : 0) << m) | jj) << N) + (unsigned)(in ? y : 0);
    const float2 v = *reinterpret_cast<const float2 *>(R + at);
    return in ? v : make_float2(e, e);
}

// One pair of rows (y, y+1) of R_n at probe column x, cone pair ii (cones
// jj = 2 ii, 2 ii + 1), FP32 intervals.  Every operand, the cone weights
// included, is loaded before any is used, so a wave waits for memory once;
// TOP (n + 1 = N) builds the doubled edges of T_N from T_{N-1} and reads the
// environment for R_N; without ENV the fluence from beyond the grid is 0 (a
// constant, so the lookups outside the grid stay selects, not branches).
// Addresses are 32-bit element offsets from the level's base (a T level of
// four quadrants holds fewer than 2^27 entries).  The arithmetic, and its
// order, is that of Eq. 14 (odd x) and Eq. 15-17 (even x).
template <bool TOP, bool ENV>
__device__ __forceinline__ float2 merge_down_pair(const DownArgs &a, int q, int x, int ii, int y) {
    const int N = a.N, S = 1 << N, n = a.n, m = n + 1;
    const unsigned rq = (unsigned)q << (2 * N);
    const int jb = (1 << m) - 1 + 2 * ii;  // cone table index of cone 2 ii at level m
    const float A0 = c_cone[jb], A1 = c_cone[jb + 1];
    float E0 = 0.f, E1 = 0.f;
    if (ENV) {
        const float *ep = a.env + (size_t)(a.q0 + q) * kConeTable + jb;
        E0 = ep[0];
        E1 = ep[1];
    }
    float acc0 = 0.f, acc1 = 0.f;
    if (x & 1) {
        // Eq. 14: the half-cone's outer edge (T_n of this column, directions
        // ii and ii + 1) to the level n+1 probe c.
        const unsigned tx = (unsigned)q * (unsigned)a.en + ((unsigned)x * ((1u << n) + 1) << N) +
                            ((unsigned)ii << N) + (unsigned)y;
        const int c = (x + 1) >> 1;
        const int yr = y + 2 * ii - (1 << n);
        const float4 t0 = ld_pair(a.Tn + tx);
        const float4 t1 = ld_pair(a.Tn + tx + S);
        float2 f0 = make_float2(E0, E0), f1 = make_float2(E1, E1);
        if (!TOP) {
            f0 = r_pair_sel(a.Rn1, rq, N, m, c, 2 * ii, yr, E0);
            f1 = r_pair_sel(a.Rn1, rq, N, m, c, 2 * ii + 1, yr + 2, E1);
        }
        acc0 += fmaf(t0.y, f0.x, A0 * t0.x);
        acc1 += fmaf(t0.w, f0.y, A0 * t0.z);
        acc0 += fmaf(t1.y, f1.x, A1 * t1.x);
        acc1 += fmaf(t1.w, f1.y, A1 * t1.z);
    } else {
        // Eq. 15-17: the co-located probe c averaged with the doubled edge
        // T_{n+1}(c, e2), e2 = 2 ii and 2 ii + 2, to probe c + 1.
        const int c = x >> 1;
        float4 t0, t1;
        if (TOP) {
            // T_N(c, e2) as the merge up builds an even direction (Eq. 18):
            // T_{N-1}(2c, e2/2) at row y, then T_{N-1}(2c+1, e2/2) at row
            // y + e2 - 2^n.
            const unsigned dn = (1u << n) + 1;
            const unsigned tn = (unsigned)q * (unsigned)a.en + ((unsigned)(2 * c) * dn << N) +
                                ((unsigned)ii << N);
            const float2 *Tnear = a.Tn + tn;
            const float2 *Tfar = Tnear + (dn << N);
            const float4 nv0 = ld_pair(Tnear + y);
            const float4 nv1 = ld_pair(Tnear + S + y);
            const float4 fv0 = far_pair_sel(Tfar, y + 2 * ii - (1 << n), S);
            const float4 fv1 = far_pair_sel(Tfar + S, y + 2 * ii + 2 - (1 << n), S);
            t0 = pair(merge(lo(nv0), lo(fv0)), merge(hi(nv0), hi(fv0)));
            t1 = pair(merge(lo(nv1), lo(fv1)), merge(hi(nv1), hi(fv1)));
        } else {
            const unsigned tx = (unsigned)q * (unsigned)a.en1 + ((unsigned)c * ((1u << m) + 1) << N) +
                                ((unsigned)(2 * ii) << N) + (unsigned)y;
            t0 = ld_pair(a.Tn1 + tx);
            t1 = ld_pair(a.Tn1 + tx + 2 * S);
        }
        float2 r00 = make_float2(E0, E0), r01 = make_float2(E1, E1);
        float2 r10 = r00, r11 = r01;
        if (!TOP) {
            const int yf = y + 4 * ii - (1 << m);
            r00 = r_pair_sel(a.Rn1, rq, N, m, c, 2 * ii, y, E0);
            r01 = r_pair_sel(a.Rn1, rq, N, m, c, 2 * ii + 1, y, E1);
            r10 = r_pair_sel(a.Rn1, rq, N, m, c + 1, 2 * ii, yf, E0);
            r11 = r_pair_sel(a.Rn1, rq, N, m, c + 1, 2 * ii + 1, yf + 4, E1);
        }
        acc0 += 0.5f * (r00.x + fmaf(t0.y, r10.x, A0 * t0.x));
        acc1 += 0.5f * (r00.y + fmaf(t0.w, r10.y, A0 * t0.z));
        acc0 += 0.5f * (r01.x + fmaf(t1.y, r11.x, A1 * t1.x));
        acc1 += 0.5f * (r01.y + fmaf(t1.w, r11.y, A1 * t1.z));
    }
    return make_float2(acc0, acc1);
}

// R_{n+1} at (c, jj) for rows y .. y+3, y a multiple of 4 (so the four are in
// or out of the grid together), or the environment's fluence e outside it: a
// clamped address and a select.
__device__ __forceinline__ float4 r_quad_sel(const float *R, unsigned rq, int N, int m, int c,
                                             int jj, int y, float e) {
    const int S = 1 << N;
    const bool in = c < (S >> m) && (unsigned)y < (unsigned)S;
    const unsigned at = rq + ((unsigned)(((in ? c : 0) << m) | jj) << N) + (unsigned)(in ? y : 0);
    const float4 v = *reinterpret_cast<const float4 *>(R + at);
    return in ? v : make_float4(e, e, e, e);
}

// The 16-bit form of merge_down_pair: rows y .. y+3 (y a multiple of 4) of
// R_n, each T row read as one quad of intervals, and every operand loaded
// before any is used.  Lookups whose row shift is only even (Eq. 14, and the
// far end of T_N's doubled edges) take two pairs, each with its own select.
template <bool TOP, bool ENV>
__device__ __forceinline__ float4 merge_down_quad(const DownArgs &a, int q, int x, int ii, int y) {
    const int N = a.N, S = 1 << N, n = a.n, m = n + 1;
    const unsigned rq = (unsigned)q << (2 * N);
    const half2_t *Tn = reinterpret_cast<const half2_t *>(a.Tn);
    const half2_t *Tn1 = reinterpret_cast<const half2_t *>(a.Tn1);
    const int jb = (1 << m) - 1 + 2 * ii;
    const float A[2] = {c_cone[jb], c_cone[jb + 1]};
    float E[2] = {0.f, 0.f};
    if (ENV) {
        const float *ep = a.env + (size_t)(a.q0 + q) * kConeTable + jb;
        E[0] = ep[0];
        E[1] = ep[1];
    }
    float acc0[2] = {0.f, 0.f}, acc1[2] = {0.f, 0.f};
    if (x & 1) {
        // Eq. 14
        const unsigned tx = (unsigned)q * (unsigned)a.en + ((unsigned)x * ((1u << n) + 1) << N) +
                            ((unsigned)ii << N) + (unsigned)y;
        const int c = (x + 1) >> 1;
        const int yr = y + 2 * ii - (1 << n);
        half8_t h[2];
        float2 rf[2][2];
#pragma unroll
        for (int up = 0; up < 2; ++up) {
            h[up] = *reinterpret_cast<const half8_t *>(Tn + tx + up * S);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                rf[up][j] = TOP ? make_float2(E[up], E[up])
                                : r_pair_sel(a.Rn1, rq, N, m, c, 2 * ii + up, yr + 2 * up + 2 * j, E[up]);
        }
#pragma unroll
        for (int up = 0; up < 2; ++up) {
            pin(h[up]);
            float4 t[2];
            cvt_quad(h[up], t[0], t[1]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc0[j] += fmaf(t[j].y, rf[up][j].x, A[up] * t[j].x);
                acc1[j] += fmaf(t[j].w, rf[up][j].y, A[up] * t[j].z);
            }
        }
    } else {
        // Eq. 15-17
        const int c = x >> 1;
        float4 t[2][2];
        if (TOP) {
            const unsigned dn = (1u << n) + 1;
            const unsigned tn = (unsigned)q * (unsigned)a.en + ((unsigned)(2 * c) * dn << N) +
                                ((unsigned)ii << N);
            half8_t hn[2];
            half4_t hf[2][2];
            bool in[2][2];
#pragma unroll
            for (int up = 0; up < 2; ++up) {
                const half2_t *near = Tn + tn + up * S, *far = near + (dn << N);
                const int yf = y + 2 * ii + 2 * up - (1 << n);
                hn[up] = *reinterpret_cast<const half8_t *>(near + y);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    in[up][j] = (unsigned)(yf + 2 * j) < (unsigned)S;
                    hf[up][j] = *reinterpret_cast<const half4_t *>(far + (in[up][j] ? yf + 2 * j : 0));
                }
            }
#pragma unroll
            for (int up = 0; up < 2; ++up) {
                pin(hn[up]);
                float4 nv[2];
                cvt_quad(hn[up], nv[0], nv[1]);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    pin(hf[up][j]);
                    const half4_t v = hf[up][j];
                    const float4 fv = in[up][j] ? make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w)
                                                : make_float4(0.f, 1.f, 0.f, 1.f);
                    t[up][j] = pair(merge(lo(nv[j]), lo(fv)), merge(hi(nv[j]), hi(fv)));
                }
            }
        } else {
            const unsigned tx = (unsigned)q * (unsigned)a.en1 + ((unsigned)c * ((1u << m) + 1) << N) +
                                ((unsigned)(2 * ii) << N) + (unsigned)y;
            half8_t h[2];
#pragma unroll
            for (int up = 0; up < 2; ++up) h[up] = *reinterpret_cast<const half8_t *>(Tn1 + tx + 2 * up * S);
#pragma unroll
            for (int up = 0; up < 2; ++up) {
                pin(h[up]);
                cvt_quad(h[up], t[up][0], t[up][1]);
            }
        }
        float4 r0[2], r1[2];
#pragma unroll
        for (int up = 0; up < 2; ++up) {
            const float e = E[up];
            r0[up] = r1[up] = make_float4(e, e, e, e);
            if (!TOP) {
                r0[up] = r_quad_sel(a.Rn1, rq, N, m, c, 2 * ii + up, y, e);
                r1[up] = r_quad_sel(a.Rn1, rq, N, m, c + 1, 2 * ii + up, y + 4 * ii + 4 * up - (1 << m), e);
            }
        }
#pragma unroll
        for (int up = 0; up < 2; ++up) {
            const float2 ra[2] = {make_float2(r0[up].x, r0[up].y), make_float2(r0[up].z, r0[up].w)};
            const float2 rb[2] = {make_float2(r1[up].x, r1[up].y), make_float2(r1[up].z, r1[up].w)};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc0[j] += 0.5f * (ra[j].x + fmaf(t[up][j].y, rb[j].x, A[up] * t[up][j].x));
                acc1[j] += 0.5f * (ra[j].y + fmaf(t[up][j].w, rb[j].y, A[up] * t[up][j].z));
            }
        }
    }
    return make_float4(acc0[0], acc1[0], acc0[1], acc1[1]);
}

// Merge down: R_n from R_{n+1}, T_n, T_{n+1} (Eq. 14-17), for n >= 1 (levels 1
// and 0 of the forward are the tail's, and the reverse reads R_1 at the
// lowest), so every row shift is even and each lookup is a pair.
template <typename TS>
__device__ void body_merge_down(const DownArgs &a, unsigned tile, int U, int tid) {
    constexpr int P = merge_pairs<TS>();
    const int N = a.N, S = 1 << N, n = a.n;
    const size_t SS = (size_t)S * S;
    const size_t total = (size_t)a.nq * (SS / (2 * P));
    const int m = n + 1;
    for (int uu = 0; uu < U; ++uu) {
        const size_t idx = ((size_t)tile * U + uu) * 256 + tid;
        if (idx >= total) return;
        const int y0 = (int)(idx & (S / (2 * P) - 1)) * 2 * P;
        const unsigned row = (unsigned)(idx >> (N - (P == 2 ? 2 : 1)));
        const int q = row >> N;
        int x, ii;
        if (a.blk) {
            // rows in blocks of 2^blk directions, every probe column of a
            // block together: the columns that read the same R_{n+1} and T
            // rows run side by side on one XCD
            const unsigned rr = row & (S - 1), lb = a.blk, lx = N - n;
            x = (int)((rr >> lb) & ((1u << lx) - 1));
            ii = (int)(((rr >> (lb + lx)) << lb) | (rr & ((1u << lb) - 1)));
        } else {
            x = (int)((row & (S - 1)) >> n);
            ii = (int)(row & ((1u << n) - 1));
        }
        const unsigned r = ((unsigned)x << n) | (unsigned)ii;
        float *out = a.R + q * SS + (size_t)r * S + y0;
        if constexpr (P == 1) {
            float2 v;
            if (a.env)
                v = m == N ? merge_down_pair<true, true>(a, q, x, ii, y0)
                           : merge_down_pair<false, true>(a, q, x, ii, y0);
            else
                v = m == N ? merge_down_pair<true, false>(a, q, x, ii, y0)
                           : merge_down_pair<false, false>(a, q, x, ii, y0);
            *reinterpret_cast<float2 *>(out) = v;
        } else {
            // 16-bit intervals: rows y0 .. y0+3 per thread, each T row one quad.
            float4 v;
            if (a.env)
                v = m == N ? merge_down_quad<true, true>(a, q, x, ii, y0)
                           : merge_down_quad<false, true>(a, q, x, ii, y0);
            else
                v = m == N ? merge_down_quad<true, false>(a, q, x, ii, y0)
                           : merge_down_quad<false, false>(a, q, x, ii, y0);
            *reinterpret_cast<float4 *>(out) = v;
        }
    }
}

// Tail of the forward, per TILE x TILE image tile and every quadrant of the
// group: the merge down of levels 1 and 0 (Eq. 14-17), the gather of
// Algorithm 1 (R_0 at the probe one pixel ahead, cone 0) and the sum of the
// quadrants' gathers on the image.  For each quadrant, R_1 over the level-1
// columns and rows the tile's level-0 values read is built from R_2 into LDS,
// then R_0 one column ahead of every pixel from it.  The intervals these two
// levels read (both directions of T_0, all of T_1, the even directions of T_2)
// are folded here from the tile's pixel intervals, as the traced levels are
// built, instead of being stored and read back: they hold only axis and
// diagonal half pieces.  Quadrants are summed in order 0..3, and a later group
// adds to the sum the earlier groups stored.
template <int TILE> struct TailTile {
    // T_2 rays run 4 pixels ahead of level-1 probes up to 2 columns past the
    // tile and +-4 rows around rows up to 2 beyond it
    static constexpr int halo = 6;
    static constexpr int span = TILE + 2 * halo;
    static constexpr int pitch = span + 1;
    static constexpr int plane = span * pitch;
    static constexpr int r1cols = TILE / 2 + 1;  // level-1 columns u_lo/2 + 1 .. u_lo/2 + TILE/2 + 1
    static constexpr int r1rows = TILE + 4;      // rows w_lo - 2 .. w_lo + TILE + 1
    static constexpr int acc_pitch = TILE + 1;
    static constexpr int iv_bytes = 2 * plane * 8;
    static constexpr int r1_bytes = r1cols * 2 * r1rows * 4;
    static constexpr int lds = iv_bytes + r1_bytes + TILE * acc_pitch * 4;
};

// Fold of the half pieces of traced ray `sid` (stencil ids as in the traced
// levels) from the probe's pixel interval at ivp; su / sw step one pixel in u
// / w, and the two planes hold the axis and the diagonal half pieces.
template <int sid, int pieces, int plane, typename I>
__device__ __forceinline__ I tail_ray(const I *ivp, int su, int sw) {
    I acc = ivp[kHpLen[sid][0] * plane];  // the first piece lies in the probe's pixel
#pragma unroll
    for (int j = 1; j < pieces; ++j)
        acc = merge(acc, ivp[kHpLen[sid][j] * plane + kHpDu[sid][j] * su + kHpDw[sid][j] * sw]);
    return acc;
}

// R_2 of one quadrant at the column whose row block starts at `ro` (clamped
// into the grid by the caller), cone jj, row y: the stored value when the
// column (cin) and the row lie in the grid, else `fill`.  The load is always
// in bounds, so the lookup needs no branch.
__device__ __forceinline__ float r2_at(const float *R2, int ro, int jj, int y, int S, bool cin,
                                       float fill) {
    const bool in = cin && (unsigned)y < (unsigned)S;
    const float v = R2[in ? (unsigned)(ro + jj * S + y) : 0u];
    return in ? v : fill;
}

template <int TILE>
__device__ void body_tail(const TailArgs &a, unsigned tile, char *lds, int tid) {
    using G = TailTile<TILE>;
    constexpr int H = G::halo, P = G::pitch, RR = G::r1rows, AP = G::acc_pitch;
    constexpr int span2 = G::span * G::span;
    float2 *iv = reinterpret_cast<float2 *>(lds);
    float *r1 = reinterpret_cast<float *>(lds + G::iv_bytes);
    float *acc = reinterpret_cast<float *>(lds + G::iv_bytes + G::r1_bytes);
    const int N = a.N, S = 1 << N;
    const int tiles = (S + TILE - 1) / TILE;
    const int r0 = (int)(tile / tiles) * TILE, c0 = (int)(tile % tiles) * TILE;
#pragma unroll
    for (int it = 0; it < (span2 + 255) / 256; ++it) {
        const int i = tid + 256 * it;
        if (i < span2) {
            const int lr = i / G::span, lc = i % G::span;
            const int r = r0 - H + lr, c = c0 - H + lc;
            const bool in = (unsigned)r < (unsigned)S && (unsigned)c < (unsigned)S;
            const int off = in ? r * S + c : 0;
            const float e = a.eps[off], g = a.sig[off];
            iv[lr * P + lc] = cell_interval(in ? e : 0.f, in ? g : 0.f, 0.5f);
            iv[G::plane + lr * P + lc] = cell_interval(in ? e : 0.f, in ? g : 0.f, kH2);
        }
    }
#pragma unroll
    for (int it = 0; it < TILE * TILE / 256; ++it) {
        const int i = tid + 256 * it;
        const int rl = i / TILE, cl = i % TILE;
        const int r = r0 + rl, c = c0 + cl;
        acc[rl * AP + cl] = (a.accumulate && r < S && c < S) ? a.out[r * S + c] : 0.f;
    }
    for (int g = 0; g < a.nq; ++g) {
        const int q = a.q0 + g;
        const float *R2 = a.R2 + (size_t)g * S * S;
        const float *envq = a.env ? a.env + (size_t)q * kConeTable : nullptr;
        // angular fluences beyond the grid (uniform over the tile)
        const float e10 = env_fluence(envq, 1, 0), e11 = env_fluence(envq, 1, 1);
        const float e20 = env_fluence(envq, 2, 0), e21 = env_fluence(envq, 2, 1);
        const float e22 = env_fluence(envq, 2, 2), e23 = env_fluence(envq, 2, 3);
        // frame of quadrant q: +x (u, w) = (c, r); -x (S-1-c, r); +y (r, c); -y (S-1-r, c);
        // the tile covers u_lo .. u_lo + TILE - 1, w_lo .. w_lo + TILE - 1, and
        // frame pixel (u, w) sits at LDS index base + (u - u_lo) su + (w - w_lo) sw
        const int u_lo = q == 0 ? c0 : q == 1 ? S - TILE - c0 : q == 2 ? r0 : S - TILE - r0;
        const int w_lo = q < 2 ? r0 : c0;
        const int su = q == 0 ? 1 : q == 1 ? -1 : q == 2 ? P : -P;
        const int sw = q < 2 ? P : 1;
        const int base = q == 1 ? H * P + TILE - 1 + H : q == 3 ? (TILE - 1 + H) * P + H : H * P + H;
        const int c1_lo = u_lo / 2 + 1;  // u_lo is even, so the first level-1 column is odd
        const int cmax = S >> 2;          // level-2 columns in the grid
        __syncthreads();  // intervals and sums in place; the previous quadrant's R_1 consumed
        // R_1 at odd level-1 columns (Eq. 14 at level 1, through T_1)
        constexpr int n_odd = (TILE / 4 + 1) * RR;
#pragma unroll
        for (int it = 0; it < (n_odd + 255) / 256; ++it) {
            const int i = tid + 256 * it;
            if (i >= n_odd) break;
            const int j = 2 * (i / RR), wl = i % RR;
            const int cp = c1_lo + j, w = w_lo - 2 + wl;
            float v0 = e10, v1 = e11;
            if (cp < 0) {
                v0 = v1 = 0.f;
            } else if (cp < (S >> 1) && (unsigned)w < (unsigned)S) {
                const float2 *ivp = iv + base + (2 * cp - u_lo) * su + (w - w_lo) * sw;
                const float2 t0 = tail_ray<2, 4, G::plane>(ivp, su, sw);
                const float2 t1 = tail_ray<3, 4, G::plane>(ivp, su, sw);
                const float2 t2 = tail_ray<4, 4, G::plane>(ivp, su, sw);
                const int c = (cp + 1) >> 1;
                const bool cin = c < cmax;
                const int ro = (cin ? c : 0) * 4 * S;
                v0 = fmaf(t0.y, r2_at(R2, ro, 0, w - 2, S, cin, e20), c_cone[3] * t0.x) +
                     fmaf(t1.y, r2_at(R2, ro, 1, w, S, cin, e21), c_cone[4] * t1.x);
                v1 = fmaf(t1.y, r2_at(R2, ro, 2, w, S, cin, e22), c_cone[5] * t1.x) +
                     fmaf(t2.y, r2_at(R2, ro, 3, w + 2, S, cin, e23), c_cone[6] * t2.x);
            }
            r1[(2 * j) * RR + wl] = v0;
            r1[(2 * j + 1) * RR + wl] = v1;
        }
        // R_1 at even level-1 columns (Eq. 15-17 at level 1, through the even directions of T_2)
        constexpr int n_even = (TILE / 4) * RR;
#pragma unroll
        for (int it = 0; it < (n_even + 255) / 256; ++it) {
            const int i = tid + 256 * it;
            if (i >= n_even) break;
            const int j = 2 * (i / RR) + 1, wl = i % RR;
            const int cp = c1_lo + j, w = w_lo - 2 + wl;
            float v0 = e10, v1 = e11;
            if (cp < 0) {
                v0 = v1 = 0.f;
            } else if (cp < (S >> 1) && (unsigned)w < (unsigned)S) {
                const float2 *ivp = iv + base + (2 * cp - u_lo) * su + (w - w_lo) * sw;
                const float2 t0 = tail_ray<5, 8, G::plane>(ivp, su, sw);
                const float2 t2 = tail_ray<7, 8, G::plane>(ivp, su, sw);
                const float2 t4 = tail_ray<9, 8, G::plane>(ivp, su, sw);
                const int c = cp >> 1;  // < cmax: cp < S / 2
                const bool cin = c + 1 < cmax;
                const int ro = c * 4 * S, ro1 = (cin ? c + 1 : 0) * 4 * S;
                v0 = 0.5f * (r2_at(R2, ro, 0, w, S, true, e20) +
                             fmaf(t0.y, r2_at(R2, ro1, 0, w - 4, S, cin, e20), c_cone[3] * t0.x)) +
                     0.5f * (r2_at(R2, ro, 1, w, S, true, e21) +
                             fmaf(t2.y, r2_at(R2, ro1, 1, w, S, cin, e21), c_cone[4] * t2.x));
                v1 = 0.5f * (r2_at(R2, ro, 2, w, S, true, e22) +
                             fmaf(t2.y, r2_at(R2, ro1, 2, w, S, cin, e22), c_cone[5] * t2.x)) +
                     0.5f * (r2_at(R2, ro, 3, w, S, true, e23) +
                             fmaf(t4.y, r2_at(R2, ro1, 3, w + 4, S, cin, e23), c_cone[6] * t4.x));
            }
            r1[(2 * j) * RR + wl] = v0;
            r1[(2 * j + 1) * RR + wl] = v1;
        }
        __syncthreads();
        // R_0 at x = u + 1 for every pixel (u, w) of the tile, added to the sum.
        // A thread keeps its row w; its column offsets ul are all even (x
        // odd) in the first half of the passes and all odd in the second, so
        // each pass holds one parity of x for the whole block (with a single
        // pass, for each wave).  Offsets into the intervals and the sum are
        // linear in ul and wl.
        constexpr int SP = 256 / TILE, IT = TILE * TILE / 256;
        const int wl = tid % TILE, w = w_lo + wl, slot0 = tid / TILE;
        const int au = q == 0 ? 1 : q == 1 ? -1 : q == 2 ? AP : -AP;
        const int aw = q < 2 ? AP : 1;
        const int abase = q == 1 ? TILE - 1 : q == 3 ? (TILE - 1) * AP : 0;
        const float2 *ivw = iv + base + su + wl * sw;  // pixel (u_lo + 1, w)
        float *accw = acc + abase + wl * aw;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int ul;
            if constexpr (IT >= 2)
                ul = 2 * (slot0 + SP * (it % (IT / 2))) + (it >= IT / 2 ? 1 : 0);
            else
                ul = slot0 < SP / 2 ? 2 * slot0 : 2 * (slot0 - SP / 2) + 1;
            const int u = u_lo + ul;
            if (u < 0 || u >= S || w >= S) continue;
            const float2 *ivp = ivw + ul * su;  // the probe at x = u + 1
            float v;
            if ((ul & 1) == 0) {
                // x odd, Eq. 14 at level 0: both directions of T_0, R_1 at the
                // next level-1 probe (column (x + 1) / 2)
                const float2 t0 = tail_ray<0, 2, G::plane>(ivp, su, sw);
                const float2 t1 = tail_ray<1, 2, G::plane>(ivp, su, sw);
                const float *rj = r1 + ul * RR + wl;
                v = fmaf(t0.y, rj[1], c_cone[1] * t0.x) + fmaf(t1.y, rj[RR + 3], c_cone[2] * t1.x);
            } else if (u + 1 < S) {
                // x even, Eq. 15-17 at level 0: the co-located level-1 probe
                // (column x / 2) and the doubled edges (directions 0 and 2 of T_1)
                const float2 t0 = tail_ray<2, 4, G::plane>(ivp, su, sw);
                const float2 t2 = tail_ray<4, 4, G::plane>(ivp, su, sw);
                const float *rj = r1 + (ul - 1) * RR + wl;
                v = 0.5f * (rj[2] + fmaf(t0.y, rj[2 * RR], c_cone[1] * t0.x)) +
                    0.5f * (rj[RR + 2] + fmaf(t2.y, rj[3 * RR + 4], c_cone[2] * t2.x));
            } else {
                v = env_fluence(envq, 0, 0);  // x = S: beyond the grid
            }
            accw[ul * au] += v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < TILE * TILE / 256; ++it) {
        const int i = tid + 256 * it;
        const int rl = i / TILE, cl = i % TILE;
        const int r = r0 + rl, c = c0 + cl;
        if (r < S && c < S) a.out[r * S + c] = acc[rl * AP + cl];
    }
    __syncthreads();
}

// Transpose of the gather: dR_0[q][x][y] = dF at the image pixel of frame
// point (x - 1, y), and 0 at x = 0.  Tile = q * tiles^2 + (x tile, y tile).
constexpr int kGatherAdjLds = 32 * 33 * 4;

__device__ void body_gather_adj(const GatherAdjArgs &a, unsigned tile, char *lds, int tid) {
    float (*ga_tile)[33] = reinterpret_cast<float (*)[33]>(lds);
    const int N = a.N, S = 1 << N;
    const size_t SS = (size_t)S * S;
    const int tiles = (S + 31) >> 5;
    const int q = tile / (tiles * tiles);
    const int t2 = tile % (tiles * tiles);
    const int tX = t2 / tiles, tY = t2 % tiles;
    const int tx = tid & 31, ty = tid >> 5;
    // Every thread reaches both barriers whatever its tile (tiles of other
    // passes may share the block); tiles past the four quadrants store nothing.
    // The four loads of a thread are issued before any is used: positions
    // without a source read a clamped address and take 0 by a select.
    if (q == 2 || q == 3) {
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = tX * 32 + ty + 8 * i, y = tY * 32 + tx;
            const bool src = x >= 1 && x < S && y < S;
            v[i] = a.dF[(size_t)frame_row(q, src ? x - 1 : 0, S) * S + (src ? y : 0)];
            v[i] = src ? v[i] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = tX * 32 + ty + 8 * i, y = tY * 32 + tx;
            if (x < S && y < S) a.dR0[q * SS + (size_t)x * S + y] = v[i];
        }
    } else if (q < 2) {
        // +-x: frame (u, w) is image (w, u or S-1-u): read image rows w = y.
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int y = tY * 32 + ty + 8 * i, x = tX * 32 + tx;
            const bool src = x >= 1 && x < S && y < S;
            v[i] = a.dF[(size_t)(src ? y : 0) * S + frame_row(q, src ? x - 1 : 0, S)];
            v[i] = src ? v[i] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) ga_tile[ty + 8 * i][tx] = v[i];
    }
    __syncthreads();
    if (q < 2) {
        for (int i = 0; i < 4; ++i) {
            int xl = ty + 8 * i;
            int x = tX * 32 + xl, y = tY * 32 + tx;
            if (x < S && y < S) a.dR0[q * SS + (size_t)x * S + y] = ga_tile[tx][xl];
        }
    }
    __syncthreads();
}

// R at (row, y) and (row, y+1), the row starting at element `row` of `base`
// (32-bit offsets), when the row lies in the grid (`in`, uniform
// over the wave); rows y outside [0, S) and every element of a row outside the
// grid read `fill` (the environment's fluence for the cone, or 0).  With
// `even` (every shift but those of level 0) y is even and the two form one
// aligned pair.  Rows outside [0, S) load a clamped address and are replaced
// by a select, so the lookup has no per-lane branch.
__device__ __forceinline__ float2 ld2_r_at(bool in, const float *base, unsigned row, int y, int S,
                                           bool even, float fill) {
    if (!in) return make_float2(fill, fill);
    if (even) {
        const bool ok = (unsigned)y < (unsigned)S;
        const float2 v = *reinterpret_cast<const float2 *>(base + (row + (unsigned)(ok ? y : 0)));
        return ok ? v : make_float2(fill, fill);
    }
    const bool ok0 = (unsigned)y < (unsigned)S, ok1 = (unsigned)(y + 1) < (unsigned)S;
    const float a0 = base[row + (unsigned)(ok0 ? y : 0)], a1 = base[row + (unsigned)(ok1 ? y + 1 : 0)];
    return make_float2(ok0 ? a0 : fill, ok1 ? a1 : fill);
}

// Adjoint of the merge down: dR_{n+1} from dR_n (gather form).  Each R_{n+1}
// entry (c, jj, y') is read by at most three R_n entries: the odd column 2c-1
// (far end of Eq. 14), the even column 2c (F^0 of Eq. 16) and the even column
// 2c-2 (far end of Eq. 17).  Two consecutive y' per thread.
template <typename TS>
__device__ void body_merge_down_adj(const DownAdjArgs &a, unsigned tile, int U, int tid) {
    const int N = a.N, S = 1 << N, n = a.n, m = n + 1;
    const size_t SS = (size_t)S * S;
    for (int uu = 0; uu < U; ++uu) {
        const size_t idx = ((size_t)tile * U + uu) * 256 + tid;
        if (idx >= 2 * SS) return;
        const int yp = (int)(idx & (S / 2 - 1)) * 2;
        const unsigned row = (unsigned)(idx >> (N - 1));
        const int q = row >> N;
        const unsigned r = row & (S - 1);
        const int c = r >> m, jj = r & ((1 << m) - 1);
        const int ii = jj >> 1, up = jj & 1;
        const unsigned qS = (unsigned)q << (2 * N);  // 32-bit element offsets
        // Every operand is loaded before any is used (one memory wait per
        // wave); c >= 1 and n > 0 are uniform over the wave, and rows outside
        // the grid take a clamped address and a select.
        const float2 f0 = *reinterpret_cast<const float2 *>(
            a.dR + (qS + ((unsigned)(((2 * c) << n) | ii) << N) + (unsigned)yp));
        float2 g = make_float2(0.f, 0.f), t = make_float2(0.f, 0.f);
        float2 g2 = make_float2(0.f, 0.f), t2 = make_float2(0.f, 0.f);
        if (c >= 1) {
            // odd column 2c-1 (far end of Eq. 14) at row y = y' - (2e - 2^n)
            const int e = ii + up;
            const int x = 2 * c - 1;
            const int y = yp - (2 * e - (1 << n));  // odd when n = 0
            const float *grow = a.dR + (qS + ((unsigned)((x << n) | ii) << N));
            const TS *trow = reinterpret_cast<const TS *>(a.Tn) +
                             ((unsigned)q * (unsigned)a.en + ((unsigned)(x * ((1 << n) + 1) + e) << N));
            if (n > 0) {
                const bool in = (unsigned)y < (unsigned)S;
                const int yc = in ? y : 0;
                const float2 gv = *reinterpret_cast<const float2 *>(grow + yc);
                const float4 tv = ld_pair(trow + yc);
                g = in ? gv : make_float2(0.f, 0.f);
                t = in ? make_float2(tv.y, tv.w) : make_float2(0.f, 0.f);
            } else {
                const bool in0 = (unsigned)y < (unsigned)S, in1 = (unsigned)(y + 1) < (unsigned)S;
                const int y0 = in0 ? y : 0, y1 = in1 ? y + 1 : 0;
                const float ga = grow[y0], gb = grow[y1];
                const float ta = iv_t(trow + y0), tb = iv_t(trow + y1);
                g = make_float2(in0 ? ga : 0.f, in1 ? gb : 0.f);
                t = make_float2(in0 ? ta : 0.f, in1 ? tb : 0.f);
            }
            // even column 2c-2 (far end of Eq. 17) at row y' - (2 e2 - 2^(n+1))
            const int e2 = 2 * ii + 2 * up;
            const int x2 = 2 * c - 2;
            const int y2 = yp - (2 * e2 - (1 << m));
            const bool in2 = (unsigned)y2 < (unsigned)S;
            const int y2c = in2 ? y2 : 0;
            const float2 g2v = *reinterpret_cast<const float2 *>(
                a.dR + (qS + ((unsigned)((x2 << n) | ii) << N) + (unsigned)y2c));
            const float4 t2v = ld_pair(reinterpret_cast<const TS *>(a.Tn1) +
                                       ((unsigned)q * (unsigned)a.en1 +
                                        ((unsigned)((c - 1) * ((1 << m) + 1) + e2) << N) + (unsigned)y2c));
            g2 = in2 ? g2v : make_float2(0.f, 0.f);
            t2 = in2 ? make_float2(t2v.y, t2v.w) : make_float2(0.f, 0.f);
        }
        float acc0 = 0.5f * f0.x, acc1 = 0.5f * f0.y;
        acc0 = fmaf(g.x, t.x, acc0);
        acc1 = fmaf(g.y, t.y, acc1);
        acc0 = fmaf(0.5f * g2.x, t2.x, acc0);
        acc1 = fmaf(0.5f * g2.y, t2.y, acc1);
        *reinterpret_cast<float2 *>(a.dRn1 + (qS + (r << N) + (unsigned)yp)) = make_float2(acc0, acc1);
    }
}

// Adjoint of the interval pyramid: dT_n (gather form) from the merge down at
// levels n and n-1 and from the merge up of T_{n+1}.  Two consecutive y per
// thread.  Every operand is loaded first and the terms are added afterwards,
// so that a wave waits for memory once rather than once per source: the
// conditions on x and k are uniform over the wave, absent terms load nothing
// and add zero, and reads outside the grid take a clamped address and a select.
// Without ENV the fluence from beyond the grid is the constant 0, which keeps
// those selects from turning into branches that wait on the environment table.
template <typename TS, bool ENV>
__device__ __forceinline__ void dT_output(const DTArgs &a, int q, int x, int k, int y) {
    const int N = a.N, S = 1 << N, n = a.n;
    const int dirs = (1 << n) + 1;
    const unsigned r = (unsigned)(x * dirs + k);
    const float *envq = ENV ? a.env + (size_t)q * kConeTable : nullptr;
    // element offsets within each level are 32-bit (a level of four
    // quadrants holds fewer than 2^28 entries)
    const unsigned qS = (unsigned)q << (2 * N);
    // (a) merge down at level n, odd x (Eq. 14): T_n(p, k) is the edge of
    //     cone k (lower half, jj = 2k) and of cone k-1 (upper half, jj = 2k-1):
    //     term i = 0 reads R_n row (x, k-1) and cone 2k-1 of R_{n+1}, i = 1
    //     row (x, k) and cone 2k.
    float2 ag[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    float2 ar[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    float aA[2] = {0.f, 0.f};
    if (n < N && (x & 1)) {
        const int c = (x + 1) >> 1, yf = y + 2 * k - (1 << n);  // odd when n = 0
        const bool rin = n + 1 < N && c < (S >> (n + 1));
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int ii = k - 1 + i, jj = 2 * k - 1 + i;
            if (ii < 0 || ii >= (1 << n)) continue;
            ag[i] = *reinterpret_cast<const float2 *>(
                a.dRn + (qS + ((unsigned)((x << n) | ii) << N) + (unsigned)y));
            aA[i] = c_cone[(1 << (n + 1)) - 1 + jj];
            ar[i] = ld2_r_at(rin, a.Rn1, qS + ((unsigned)((c << (n + 1)) | jj) << N), yf, S,
                             n > 0, env_fluence(envq, n + 1, jj));
        }
    }
    // (b) merge down at level n-1, even column 2x (Eq. 17): T_n(p, k), k even,
    //     is the doubled edge of cone k/2 (jj = k) and of cone k/2-1 (jj = k-1):
    //     term i = 0 reads dR_{n-1} row (2x, k/2-1) and cone k-1 of R_n at
    //     column x+1, i = 1 row (2x, k/2) and cone k.
    float2 bg[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    float2 br[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    float bA[2] = {0.f, 0.f};
    if (n >= 1 && (k & 1) == 0) {
        const int nm = n - 1;
        const int yf = y + 2 * k - (1 << n);
        const int xm = 2 * x;
        const bool rin = n < N && x + 1 < (S >> n);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int jj = k - 1 + i;
            if (jj < 0 || jj >= (1 << n)) continue;
            bg[i] = *reinterpret_cast<const float2 *>(
                a.dRm + (qS + ((unsigned)((xm << nm) | (k / 2 - 1 + i)) << N) + (unsigned)y));
            bA[i] = c_cone[(1 << n) - 1 + jj];
            br[i] = ld2_r_at(rin, a.Rn, qS + ((unsigned)(((x + 1) << n) | jj) << N), yf, S, true,
                             env_fluence(envq, n, jj));
        }
    }
    // (c) merge up of T_{n+1} from T_n (Eq. 18-20), H = 2^n (n >= 2: even
    //     shifts).  Outputs ko = 2k (weight 1), 2k+1 and 2k-1 (weight 1/2):
    //     near role (x even): the far partner kb = k, k+1, k-1 at row y + 2k - H;
    //     far role (x odd): the near partner ka = k, k+1, k-1, each from
    //     output row y - (2 ka - H).
    //     Both roles load one partner interval pair and one dT_{n+1} pair
    //     per output; the role only moves the rows and the fill.
    float4 cg[3], cf[3];
    float cw[3] = {0.f, 0.f, 0.f};
    const bool near_role = (x & 1) == 0;
    if (a.has_up) {
        const int H = 1 << n;
        const int odirs = 2 * H + 1;
        const TS *Tn = reinterpret_cast<const TS *>(a.Tn);
        const unsigned g0 = (unsigned)q * (unsigned)a.en1 + ((unsigned)((x >> 1) * odirs) << N);
        const unsigned part = (unsigned)q * (unsigned)a.en +
                              ((unsigned)((near_role ? x + 1 : x - 1) * dirs) << N);
        bool act[3], in[3];
        typename PairRaw<TS>::type cr[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const int ko = v == 0 ? 2 * k : (v == 1 ? 2 * k + 1 : 2 * k - 1);
            const int kp = v == 0 ? k : (v == 1 ? k + 1 : k - 1);
            const int yo = near_role ? y + 2 * k - H : y - (2 * kp - H);
            act[v] = ko >= 0 && ko <= 2 * H;
            in[v] = (unsigned)yo < (unsigned)S;
            const int yc = in[v] ? yo : 0;
            cr[v] = raw_zero<TS>();
            cg[v] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (act[v]) {
                cr[v] = ld_pair_raw(Tn + (part + ((unsigned)kp << N) + (unsigned)yc));
                cg[v] = ld_pair(a.dTn1 + (g0 + ((unsigned)ko << N) + (unsigned)(near_role ? y : yc)));
            }
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            pin(cr[v]);
            pin(cg[v]);
            cf[v] = cvt_pair(cr[v]);
            const float4 fill = near_role ? make_float4(0.f, 1.f, 0.f, 1.f)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
            cw[v] = act[v] ? (v == 0 ? 1.f : 0.5f) : 0.f;
            cf[v] = act[v] ? (in[v] ? cf[v] : fill) : make_float4(0.f, 1.f, 0.f, 1.f);
            cg[v] = act[v] && (in[v] || near_role) ? cg[v] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    } else {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            cg[v] = make_float4(0.f, 0.f, 0.f, 0.f);
            cf[v] = make_float4(0.f, 1.f, 0.f, 1.f);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        pin(ag[i]); pin(ar[i]); pin(aA[i]);
        pin(bg[i]); pin(br[i]); pin(bA[i]);
    }
    float gl0 = 0.f, gt0 = 0.f, gl1 = 0.f, gt1 = 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        gl0 = fmaf(ag[i].x, aA[i], gl0); gl1 = fmaf(ag[i].y, aA[i], gl1);
        gt0 = fmaf(ag[i].x, ar[i].x, gt0); gt1 = fmaf(ag[i].y, ar[i].y, gt1);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float g0x = 0.5f * bg[i].x, g0y = 0.5f * bg[i].y;
        gl0 = fmaf(g0x, bA[i], gl0); gl1 = fmaf(g0y, bA[i], gl1);
        gt0 = fmaf(g0x, br[i].x, gt0); gt1 = fmaf(g0y, br[i].y, gt1);
    }
    if (near_role) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const float4 g = cg[v], f = cf[v];
            gl0 = fmaf(cw[v], g.x, gl0);
            gt0 = fmaf(cw[v], fmaf(g.x, f.x, g.y * f.y), gt0);
            gl1 = fmaf(cw[v], g.z, gl1);
            gt1 = fmaf(cw[v], fmaf(g.z, f.z, g.w * f.w), gt1);
        }
    } else {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const float4 g = cg[v], tn = cf[v];
            gl0 = fmaf(cw[v] * g.x, tn.y, gl0);
            gt0 = fmaf(cw[v] * g.y, tn.y, gt0);
            gl1 = fmaf(cw[v] * g.z, tn.w, gl1);
            gt1 = fmaf(cw[v] * g.w, tn.w, gt1);
        }
    }
    *reinterpret_cast<float4 *>(a.dT + ((unsigned)q * (unsigned)a.en + (r << N) + (unsigned)y)) =
        make_float4(gl0, gt0, gl1, gt1);
}

template <typename TS, bool ENV>
__device__ void body_dT_t(const DTArgs &a, unsigned tile, int U, int tid) {
    const int N = a.N, S = 1 << N, n = a.n;
    const int dirs = (1 << n) + 1;
    // at the two lowest levels a thread takes the same (k, y) of both probe
    // columns 2c and 2c+1, which read the same dT_{n+1} rows of column c
    // (measured at 1024^2: 3-14% faster there, 1-2 us slower per level above)
    const bool pairs = n <= 1 && n < N;
    const unsigned cols = pairs ? (unsigned)(S >> n) / 2 : (unsigned)(S >> n);
    const unsigned rpq = cols * dirs;
    const size_t total = (size_t)4 * rpq * (S / 2);
    for (int uu = 0; uu < U; ++uu) {
        const size_t idx = ((size_t)tile * U + uu) * 256 + tid;
        if (idx >= total) return;
        const int y = (int)(idx & (S / 2 - 1)) * 2;
        const unsigned row = (unsigned)(idx >> (N - 1));
        const int q = (row >= rpq) + (row >= 2 * rpq) + (row >= 3 * rpq);
        const unsigned rc = row - (unsigned)q * rpq;
        const int c = (int)div_rows(rc, (unsigned)dirs), k = (int)(rc - (unsigned)c * dirs);
        if (pairs) {
            dT_output<TS, ENV>(a, q, 2 * c, k, y);
            dT_output<TS, ENV>(a, q, 2 * c + 1, k, y);
        } else {
            dT_output<TS, ENV>(a, q, c, k, y);
        }
    }
}

template <typename TS>
__device__ void body_dT(const DTArgs &a, unsigned tile, int U, int tid) {
    if (a.env)
        body_dT_t<TS, true>(a, tile, U, tid);
    else
        body_dT_t<TS, false>(a, tile, U, tid);
}

// phi'(tau) for phi(tau) = (1 - exp(-tau))/tau: a Taylor series near 0, where
// the closed form (tau + (1+tau) expm1(-tau))/tau^2 cancels.
__device__ __forceinline__ float cell_dphi(float tau) {
    if (tau < 0.25f) {
        return -0.5f + tau * (1.f / 3.f + tau * (-1.f / 8.f + tau * (1.f / 30.f +
               tau * (-1.f / 144.f + tau * (1.f / 840.f)))));
    }
    return (tau + (1.f + tau) * expm1f(-tau)) / (tau * tau);
}

// Adjoint of the traced levels, for all four quadrants of one 16x16 image
// tile, written straight to d eps and d sigma.  Each traced ray is the fold of
// half pieces c_1..c_m (Eq. 7), so with the prefix transmittance P_j:
//   dL/dL_j = P_j,  dL/dT_j = P_j L(c_j+1..m),  dT/dT_j = P_j T(c_j+1..m).
// Pixel p receives piece j of direction k of level n from the probe
// p - (du_j, dw_j), and that probe exists only when u - du_j is a multiple of
// 2^n: for each residue of u mod 2^n exactly two of the 2^(n+1) pieces qualify.
// Each wave therefore takes 64 pixels of one residue class of the frame u, so
// every test below is uniform over the wave, and refolds the two rays per
// direction from the interval tile in LDS (pieces relative to the pixel stay
// within 4 pixels, so the tile needs a 4-pixel halo).  Piece j adds
// dLoss/dL_j dL_j/d(eps, sigma) + dLoss/dT_j dT_j/d(eps, sigma), and the cell
// derivatives depend only on the pixel and the piece's half length, so each
// pixel sums dLoss/dL_j and dLoss/dT_j per half length over every ray of the
// four quadrants and applies the cell derivatives once at the end.
constexpr int kAdjTile = 16, kAdjHalo = 4;
constexpr int kAdjSpan = kAdjTile + 2 * kAdjHalo;     // 24
constexpr int kAdjPitch = kAdjSpan + 1;

// Half piece i of the traced ray of level n and direction k covers the pixel
// at (du, dw) from its probe's pixel: the piece midpoint lies at fraction
// (i + 1/2)/2^(n+1) of v_n(k) = (2^n, 2k - 2^n) from the probe's centre, so
// du = floor((2i + 3)/4) and dw = floor((2^(n+1) + (2i+1)(2k - 2^n))/2^(n+2)).
// The piece length is sqrt(2)/2 on diagonals (k = 0, 2^n), 1/2 on the axis
// (k = 2^(n-1)) and sqrt(5)/4 otherwise (n = 2, k = 1, 3).
__host__ __device__ constexpr int piece_du(int i) { return (2 * i + 3) >> 2; }
__host__ __device__ constexpr int piece_dw(int n, int k, int i) {
    return ((2 << n) + (2 * i + 1) * (2 * k - (1 << n))) >> (n + 2);
}
__host__ __device__ constexpr int piece_len(int n, int k) {
    return (k == 0 || k == (1 << n)) ? 1 : (2 * k == (1 << n) ? 0 : 2);
}

// The two pieces of level n that land on a pixel whose frame u has residue
// rho modulo 2^n (piece j covers u offset (2j + 3) / 4 from its probe).
__host__ __device__ constexpr int adj_piece(int n, int rho, int which) {
    if (n == 0) return which;
    if (n == 1) return rho == 0 ? (which ? 3 : 0) : (which ? 2 : 1);
    return rho == 0 ? (which ? 7 : 0) : 2 * rho - 1 + which;
}

// d(L, T)/d(eps, sigma) of one cell for the three half lengths 1/2, sqrt(2)/2,
// sqrt(5)/4 (index L), held as named scalars.
struct CellDer {
    float le0, le1, le2;  // dL/d eps
    float ls0, ls1, ls2;  // dL/d sigma
    float ts0, ts1, ts2;  // dT/d sigma
    __device__ __forceinline__ CellDer(float e, float s) {
        set(e, s, 0.5f, le0, ls0, ts0);
        set(e, s, kH2, le1, ls1, ts1);
        set(e, s, kQ5, le2, ls2, ts2);
    }
    __device__ __forceinline__ static void set(float e, float s, float ell, float &le,
                                               float &ls, float &ts) {
        const float tau = s * ell;
        le = ell * cell_phi(tau);
        ls = e * ell * ell * cell_dphi(tau);
        ts = -ell * exp_neg(tau);
    }
};

// The interval tile stays in image orientation.  The LDS offset of a frame
// displacement (du, dw) in quadrant Q, from a pointer H rows and H columns
// before the pixel, follows the frame maps +x (u, w) = (c, r), -x (S-1-c, r),
// +y (r, c), -y (S-1-r, c).
template <int Q>
__host__ __device__ constexpr int adj_lds_off(int du, int dw) {
    return Q == 0   ? (kAdjHalo + dw) * kAdjPitch + kAdjHalo + du
           : Q == 1 ? (kAdjHalo + dw) * kAdjPitch + kAdjHalo - du
           : Q == 2 ? (kAdjHalo + du) * kAdjPitch + kAdjHalo + dw
                    : (kAdjHalo - du) * kAdjPitch + kAdjHalo + dw;
}

// dLoss/dL_j and dLoss/dT_j of the pieces on one pixel, summed per half
// length index (0: 1/2, 1: sqrt(2)/2, 2: sqrt(5)/4).
struct AdjSums {
    float dl0 = 0.f, dl1 = 0.f, dl2 = 0.f;
    float dt0 = 0.f, dt1 = 0.f, dt2 = 0.f;
    template <int L>
    __device__ __forceinline__ void add(float dl, float dt) {
        if (L == 0) { dl0 += dl; dt0 += dt; }
        else if (L == 1) { dl1 += dl; dt1 += dt; }
        else { dl2 += dl; dt2 += dt; }
    }
};

// dLoss/dT of one quadrant's traced level as a buffer resource: a lane whose
// probe lies outside the grid reads at an offset past the end, which the
// hardware bounds check returns as zero, so the load needs neither a clamped
// address nor a select afterwards.
constexpr unsigned kBufferWord3 = 0x00020000u;  // raw 32-bit data, bounds checked
constexpr unsigned kOutside = 0x80000000u;      // beyond every level's byte count
__device__ __forceinline__ __amdgpu_buffer_rsrc_t dT_resource(const float2 *p, size_t entries) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2 *>(p), (short)0,
                                             (int)(entries * sizeof(float2)), (int)kBufferWord3);
}

// Direction k of level n in quadrant Q for a pixel at frame (u, w) whose u has
// residue rho modulo 2^n.  With all four known at compile time every piece
// offset in the tile is an immediate.  The two rays that put a piece on the
// pixel (their dLoss/dT loaded first) are each refolded around that piece.
// Rays whose probe lies outside the grid add 0.
template <int Q, int n, int rho, int k>
__device__ __forceinline__ void seed_adj_dir(__amdgpu_buffer_rsrc_t dTq, int S, int un, int w,
                                             int lane_off, const float2 *ivp, AdjSums &sum) {
    constexpr int dirs = (1 << n) + 1, pieces = 2 << n;
    constexpr int L = piece_len(n, k);
    constexpr int plane = kAdjSpan * kAdjPitch;
    float2 g[2];
#pragma unroll
    for (int which = 0; which < 2; ++which) {
        const int j = adj_piece(n, rho, which);
        // the probe's column (u - du_j) / 2^n is exact: u = rho (mod 2^n)
        const int cj = (piece_du(j) - (rho & ((1 << n) - 1))) >> n;
        const int dwj = piece_dw(n, k, j);
        const int pw = w - dwj;
        const bool ok = un >= cj && (unsigned)pw < (unsigned)S;
        // lane_off = ((u >> n) dirs S + w) * 8; the rest is uniform
        const unsigned off =
            ok ? (unsigned)(lane_off + ((k - cj * dirs) * S - dwj) * (int)sizeof(float2)) : kOutside;
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(dTq, off, 0, 0);
        g[which] = make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
    }
#pragma unroll
    for (int which = 0; which < 2; ++which) {
        const int j = adj_piece(n, rho, which);
        float pre = 1.f;
        float2 suf = make_float2(0.f, 1.f);
#pragma unroll
        for (int i = pieces - 1; i >= 0; --i) {
            if (i == j) continue;
            const float2 c = ivp[L * plane + adj_lds_off<Q>(piece_du(i) - piece_du(j),
                                                             piece_dw(n, k, i) - piece_dw(n, k, j))];
            if (i > j) suf = merge(c, suf);
            else pre *= c.y;
        }
        sum.add<L>(g[which].x * pre,                                     // dLoss/dL_j
                   pre * fmaf(g[which].x, suf.x, g[which].y * suf.y));   // dLoss/dT_j
    }
}

// Level n: the diagonals k = 0, 2^n, the axis k = 2^(n-1) and, at n = 2,
// k = 1, 3.
template <int Q, int n, int rho>
__device__ __forceinline__ void seed_adj_level(__amdgpu_buffer_rsrc_t dTq, int S, int u, int w,
                                               const float2 *ivp, AdjSums &sum) {
    constexpr int dirs = (1 << n) + 1;
    const int un = u >> n;
    const int lane_off = (un * dirs * S + w) * (int)sizeof(float2);
    seed_adj_dir<Q, n, rho, 0>(dTq, S, un, w, lane_off, ivp, sum);
    seed_adj_dir<Q, n, rho, (1 << n)>(dTq, S, un, w, lane_off, ivp, sum);
    if constexpr (n >= 1) seed_adj_dir<Q, n, rho, (1 << n) / 2>(dTq, S, un, w, lane_off, ivp, sum);
    if constexpr (n == 2) {
        seed_adj_dir<Q, n, rho, 1>(dTq, S, un, w, lane_off, ivp, sum);
        seed_adj_dir<Q, n, rho, 3>(dTq, S, un, w, lane_off, ivp, sum);
    }
}

// All three traced levels of quadrant Q for a pixel whose frame u is rho
// modulo 4.
template <int Q, int rho>
__device__ __forceinline__ void seed_adj_levels(const SeedAdjArgs &a, int u, int w,
                                                const float2 *ivp, AdjSums &sum) {
    const int S = 1 << a.N;
    seed_adj_level<Q, 0, 0>(dT_resource(a.dT0 + (size_t)Q * a.e0, a.e0), S, u, w, ivp, sum);
    seed_adj_level<Q, 1, rho & 1>(dT_resource(a.dT1 + (size_t)Q * a.e1, a.e1), S, u, w, ivp, sum);
    seed_adj_level<Q, 2, rho>(dT_resource(a.dT2 + (size_t)Q * a.e2, a.e2), S, u, w, ivp, sum);
}

// Quadrant Q for the pixel at image (r, c) in wave v.  Tile origins are
// multiples of 16 and S of 8, so the frame u of the wave's pixels is v modulo
// 4 in quadrants +x and +y and 3 - v in -x and -y.
template <int Q>
__device__ __forceinline__ void seed_adj_quadrant(const SeedAdjArgs &a, int v, int r, int c,
                                                  const float2 *ivp, AdjSums &sum) {
    const int S = 1 << a.N;
    const int u = Q == 0 ? c : Q == 1 ? S - 1 - c : Q == 2 ? r : S - 1 - r;
    const int w = Q < 2 ? r : c;
    switch ((Q == 0 || Q == 2) ? v : 3 - v) {
        case 0: seed_adj_levels<Q, 0>(a, u, w, ivp, sum); break;
        case 1: seed_adj_levels<Q, 1>(a, u, w, ivp, sum); break;
        case 2: seed_adj_levels<Q, 2>(a, u, w, ivp, sum); break;
        default: seed_adj_levels<Q, 3>(a, u, w, ivp, sum); break;
    }
}

// The quadrants +x and -x and the quadrants +y and -y of a pixel are summed by
// different threads; the first pair's six sums meet the second's in LDS (over
// the interval tile, once it is no longer read), rows padded against bank
// conflicts.
constexpr int kAccPitch = kAdjTile + 1;
constexpr int kAccPlane = kAdjTile * kAccPitch;
constexpr int kSeedAdjLds = 3 * kAdjSpan * kAdjPitch * 8;
static_assert(6 * kAccPlane * 4 <= kSeedAdjLds, "partial sums fit over the interval tile");

__device__ __forceinline__ void body_seed_adj(const SeedAdjArgs &a, unsigned tile, char *lds, int tid) {
    constexpr int P = kAdjPitch, plane = kAdjSpan * kAdjPitch, H = kAdjHalo;
    float2 *iv = reinterpret_cast<float2 *>(lds);
    const int S = 1 << a.N;
    const int tiles = (S + kAdjTile - 1) / kAdjTile;
    const int r0 = (int)(tile / tiles) * kAdjTile, c0 = (int)(tile % tiles) * kAdjTile;
    // the tile and its halo as three half-length intervals per cell: every
    // load of the thread first (cells outside the grid from a clamped address,
    // then 0), so the block waits for memory once
    constexpr int cells = kAdjSpan * kAdjSpan, NI = (cells + 255) / 256;
    float ev[NI], gv[NI];
    bool inside[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = tid + 256 * it;
        const int r = r0 - H + i / kAdjSpan, c = c0 - H + i % kAdjSpan;
        inside[it] = i < cells && (unsigned)r < (unsigned)S && (unsigned)c < (unsigned)S;
        const unsigned o = inside[it] ? (unsigned)(r * S + c) : 0u;
        ev[it] = a.eps[o];
        gv[it] = a.sig[o];
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        pin(ev[it]);
        pin(gv[it]);
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = tid + 256 * it;
        if (i < cells) {
            const float e = inside[it] ? ev[it] : 0.f, g = inside[it] ? gv[it] : 0.f;
            const int l = (i / kAdjSpan) * P + i % kAdjSpan;
            iv[l] = cell_interval(e, g, 0.5f);
            iv[plane + l] = cell_interval(e, g, kH2);
            iv[2 * plane + l] = cell_interval(e, g, kQ5);
        }
    }
    __syncthreads();
    const int v = tid >> 6, lane = tid & 63;
    const int i4 = v + 4 * (lane >> 4), i16 = lane & 15;
    // quadrants +x and -x (frame u along the row): wave v takes the tile
    // columns v, v+4, v+8, v+12, pixel (i16, i4)
    AdjSums sa;
    if (r0 + i16 < S && c0 + i4 < S) {
        const float2 *ivp = iv + i16 * P + i4;  // the pixel's cell is ivp[H * P + H]
        seed_adj_quadrant<0>(a, v, r0 + i16, c0 + i4, ivp, sa);
        seed_adj_quadrant<1>(a, v, r0 + i16, c0 + i4, ivp, sa);
    }
    // quadrants +y and -y (frame u down the column): wave v takes the tile
    // rows v, v+4, v+8, v+12, pixel (i4, i16)
    const int r = r0 + i4, c = c0 + i16;
    const bool in = r < S && c < S;
    AdjSums sb;
    if (in) {
        const float2 *ivp = iv + i4 * P + i16;
        seed_adj_quadrant<2>(a, v, r, c, ivp, sb);
        seed_adj_quadrant<3>(a, v, r, c, ivp, sb);
    }
    __syncthreads();
    float *x = reinterpret_cast<float *>(lds);  // [6][16][kAccPitch]
    const int la = i16 * kAccPitch + i4;
    x[la] = sa.dl0;
    x[kAccPlane + la] = sa.dl1;
    x[2 * kAccPlane + la] = sa.dl2;
    x[3 * kAccPlane + la] = sa.dt0;
    x[4 * kAccPlane + la] = sa.dt1;
    x[5 * kAccPlane + la] = sa.dt2;
    __syncthreads();
    if (in) {
        // each pixel adds the two pairs of quadrants and applies its cell
        // derivatives
        const int lb = i4 * kAccPitch + i16;
        const float dl0 = x[lb] + sb.dl0, dl1 = x[kAccPlane + lb] + sb.dl1;
        const float dl2 = x[2 * kAccPlane + lb] + sb.dl2, dt0 = x[3 * kAccPlane + lb] + sb.dt0;
        const float dt1 = x[4 * kAccPlane + lb] + sb.dt1, dt2 = x[5 * kAccPlane + lb] + sb.dt2;
        const CellDer d(a.eps[(size_t)r * S + c], a.sig[(size_t)r * S + c]);
        a.dE[(size_t)r * S + c] = fmaf(dl2, d.le2, fmaf(dl1, d.le1, dl0 * d.le0));
        a.dS[(size_t)r * S + c] =
            fmaf(dt2, d.ts2, fmaf(dl2, d.ls2, fmaf(dt1, d.ts1, fmaf(dl1, d.ls1,
                 fmaf(dt0, d.ts0, dl0 * d.ls0)))));
    }
    __syncthreads();  // the persistent kernel reuses the LDS for its next tile
}

// Cross blur of Eq. 21 on 16x16 pixel tiles: each pixel averages itself
// (weight 4) with its 4-neighbours inside the grid whose opacity
// alpha = 1 - exp(-sigma) is within `thr` of its own (weight 1 each), divided
// by the weights kept, so a neighbour that is ignored renormalises the rest.
__device__ __forceinline__ float blur_alpha(const float *sig, int S, int r, int c) {
    return -expm1f(-sig[(size_t)r * S + c]);
}
__device__ __forceinline__ bool blur_inside(int S, int r, int c) {
    return r >= 0 && r < S && c >= 0 && c < S;
}

__device__ void body_blur(const BlurArgs &a, unsigned tile, int tid) {
    const int S = 1 << a.N;
    const int tiles = (S + 15) >> 4;
    const int r = (int)(tile / tiles) * 16 + (tid >> 4), c = (int)(tile % tiles) * 16 + (tid & 15);
    if (r >= S || c >= S) return;
    const float am = blur_alpha(a.sig, S, r, c);
    float acc = 4.f * a.in[(size_t)r * S + c], wsum = 4.f;
    const int dr[4] = {-1, 1, 0, 0}, dc[4] = {0, 0, -1, 1};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = r + dr[i], cc = c + dc[i];
        if (blur_inside(S, rr, cc) && fabsf(blur_alpha(a.sig, S, rr, cc) - am) <= a.thr) {
            acc += a.in[(size_t)rr * S + cc];
            wsum += 1.f;
        }
    }
    a.out[(size_t)r * S + c] = acc / wsum;
}

// Transpose of body_blur (gather form): pixel q receives 4 g_q from itself and
// g_p from each 4-neighbour p that keeps q, with g_p = dOut_p / (4 + kept_p);
// kept_p needs the opacities around p, so each pixel reads a radius-2 diamond
// of sigma.  No dLoss/d sigma term: the kept set is piecewise constant in sigma.
__device__ __forceinline__ float blur_weight(const BlurArgs &a, int S, int r, int c, float ar) {
    // 1 / (4 + number of neighbours of (r, c) it keeps)
    float wsum = 4.f;
    const int dr[4] = {-1, 1, 0, 0}, dc[4] = {0, 0, -1, 1};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = r + dr[i], cc = c + dc[i];
        if (blur_inside(S, rr, cc) && fabsf(blur_alpha(a.sig, S, rr, cc) - ar) <= a.thr)
            wsum += 1.f;
    }
    return 1.f / wsum;
}

__device__ void body_blur_adj(const BlurArgs &a, unsigned tile, int tid) {
    const int S = 1 << a.N;
    const int tiles = (S + 15) >> 4;
    const int r = (int)(tile / tiles) * 16 + (tid >> 4), c = (int)(tile % tiles) * 16 + (tid & 15);
    if (r >= S || c >= S) return;
    const float aq = blur_alpha(a.sig, S, r, c);
    float acc = 4.f * a.in[(size_t)r * S + c] * blur_weight(a, S, r, c, aq);
    const int dr[4] = {-1, 1, 0, 0}, dc[4] = {0, 0, -1, 1};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = r + dr[i], cc = c + dc[i];
        if (!blur_inside(S, rr, cc)) continue;
        const float ap = blur_alpha(a.sig, S, rr, cc);
        if (fabsf(aq - ap) <= a.thr)
            acc += a.in[(size_t)rr * S + cc] * blur_weight(a, S, rr, cc, ap);
    }
    a.out[(size_t)r * S + c] = acc;
}

// ---------------------------------------------------------------------------
// Three radiance channels over one attenuation (RGB).  The channels see the
// same medium (Section 3: they are independent; Section 5 stores radiance as a
// 3-vector), so they share every transmittance: an interval is one float4
// (L_r, L_g, L_b, T), 16 bytes where three one-channel solves would move 24,
// and a cascade level is three planes of floats (plane c at c * nq * S^2).
// Every channel's arithmetic is that of the one-channel bodies, in the same
// order, so each channel's fluence equals the one-channel forward's bitwise.
// 16x16 image tiles (a 32x32 tile of RGB intervals would not leave LDS for
// two blocks per CU), all four quadrants at once, no environment map; the
// reverse follows the forward below.  With the 16-bit storage (the paper's: radiance and
// transmittance as halves) an interval is four halves, 8 bytes, computed in
// FP32 and rounded once when stored.
// ---------------------------------------------------------------------------

template <int TILE> struct SeedTileRgb {
    static constexpr int span = TILE + 2 * kSeedHalo;
    static constexpr int pitch = span + 1;
    static constexpr int lds = 3 * span * pitch * 16;
};

// Traced level T_2 of every quadrant (the tail folds T_0 and T_1 itself), and
// T_0, T_1 as well for the reverse's recomputed forward (a.first = 0).
template <int TILE, typename TS>
__device__ void body_seed_rgb(const SeedArgs &a, unsigned tile, char *lds, int tid) {
    using G = SeedTileRgb<TILE>;
    float4 *iv = reinterpret_cast<float4 *>(lds);
    const int S = 1 << a.N;
    const size_t SS = (size_t)S * S;
    const int tiles = (S + TILE - 1) / TILE;
    const int r0 = (int)(tile / tiles) * TILE, c0 = (int)(tile % tiles) * TILE;
    // every field load of the thread first, then the intervals (as body_seed)
    constexpr int cells = G::span * G::span, NI = (cells + 255) / 256;
    float ev[NI][3], gv[NI];
    bool inside[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = tid + 256 * it;
        const int r = r0 - kSeedHalo + i / G::span, c = c0 - kSeedHalo + i % G::span;
        inside[it] = i < cells && (unsigned)r < (unsigned)S && (unsigned)c < (unsigned)S;
        const size_t o = inside[it] ? (size_t)r * S + c : 0;
        ev[it][0] = a.eps[o];
        ev[it][1] = a.eps[SS + o];
        ev[it][2] = a.eps[2 * SS + o];
        gv[it] = a.sig[o];
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        pin(ev[it][0]);
        pin(ev[it][1]);
        pin(ev[it][2]);
        pin(gv[it]);
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = tid + 256 * it;
        if (i < cells) {
            const bool in = inside[it];
            const float e0 = in ? ev[it][0] : 0.f, e1 = in ? ev[it][1] : 0.f;
            const float e2 = in ? ev[it][2] : 0.f, g = in ? gv[it] : 0.f;
            const int l = (i / G::span) * G::pitch + i % G::span;
            iv[l] = cell_interval_rgb(e0, e1, e2, g, 0.5f);
            iv[G::span * G::pitch + l] = cell_interval_rgb(e0, e1, e2, g, kH2);
            iv[2 * G::span * G::pitch + l] = cell_interval_rgb(e0, e1, e2, g, kQ5);
        }
    }
    __syncthreads();
    for (int g = 0; g < a.nq; ++g) {
        if (a.first <= 0) seed_level_rays<TILE, 0, TS, float4>(iv, a, a.q0 + g, g, r0, c0, tid);
        if (a.first <= 1) seed_level_rays<TILE, 1, TS, float4>(iv, a, a.q0 + g, g, r0, c0, tid);
        seed_level_rays<TILE, 2, TS, float4>(iv, a, a.q0 + g, g, r0, c0, tid);
    }
    __syncthreads();
}

// Two consecutive RGB intervals of a row at y (even), or <0, 1> both when the
// row position lies outside the grid (y and S even: both in or both out).
template <typename TS>
__device__ __forceinline__ void far_pair_rgb(const TS *row, int yf, int S, float4 &a, float4 &b) {
    if (yf >= 0 && yf < S) {
        a = ld4(row + yf);
        b = ld4(row + yf + 1);
    } else {
        a = b = empty_interval<float4>();
    }
}

__device__ __forceinline__ float4 mean4(float4 p, float4 m) {
    return make_float4(0.5f * (p.x + m.x), 0.5f * (p.y + m.y), 0.5f * (p.z + m.z),
                       0.5f * (p.w + m.w));
}

// Merge up (Eq. 18-20) of RGB intervals, two consecutive y per thread.
template <typename TS>
__device__ void body_merge_up_rgb(const UpArgs &a, unsigned tile, int U, int tid) {
    const int N = a.N, S = 1 << N, n = a.n;
    const int h = 1 << (n - 1);
    const int dirs = 2 * h + 1, pdirs = h + 1;
    const unsigned rpq = (unsigned)(S >> n) * dirs;
    const size_t total = (size_t)a.nq * rpq * (S / 2);
    for (int uu = 0; uu < U; ++uu) {
        const size_t idx = ((size_t)tile * U + uu) * 256 + tid;
        if (idx >= total) return;
        const int y = (int)(idx & (S / 2 - 1)) * 2;
        const unsigned row = (unsigned)(idx >> (N - 1));
        const int q = (row >= rpq) + (row >= 2 * rpq) + (row >= 3 * rpq);
        const unsigned rk = row - (unsigned)q * rpq;
        const int x = (int)div_rows(rk, (unsigned)dirs), k = (int)(rk - (unsigned)x * dirs);
        const unsigned r = rk;
        const TS *near = reinterpret_cast<const TS *>(a.Tp) +
                         ((unsigned)q * (unsigned)a.ep + ((unsigned)(2 * x) * pdirs << N));
        const TS *far = near + ((unsigned)pdirs << N);
        float4 o0, o1;
        if ((k & 1) == 0) {
            const int kk = k >> 1;
            const float4 n0 = ld4(near + (size_t)kk * S + y), n1 = ld4(near + (size_t)kk * S + y + 1);
            float4 f0, f1;
            far_pair_rgb(far + (size_t)kk * S, y + 2 * kk - h, S, f0, f1);
            o0 = merge(n0, f0);
            o1 = merge(n1, f1);
        } else {
            const int ka = (k + 1) >> 1, kb = (k - 1) >> 1;
            const float4 na0 = ld4(near + (size_t)ka * S + y), na1 = ld4(near + (size_t)ka * S + y + 1);
            const float4 nb0 = ld4(near + (size_t)kb * S + y), nb1 = ld4(near + (size_t)kb * S + y + 1);
            float4 fa0, fa1, fb0, fb1;
            far_pair_rgb(far + (size_t)kb * S, y + 2 * ka - h, S, fa0, fa1);
            far_pair_rgb(far + (size_t)ka * S, y + 2 * kb - h, S, fb0, fb1);
            o0 = mean4(merge(na0, fa0), merge(nb0, fb0));
            o1 = mean4(merge(na1, fa1), merge(nb1, fb1));
        }
        TS *out = reinterpret_cast<TS *>(a.T) + q * a.e + (size_t)r * S + y;
        st_iv(out, o0);
        st_iv(out + 1, o1);
    }
}

__device__ __forceinline__ float chan(float4 v, int c) { return c == 0 ? v.x : c == 1 ? v.y : v.z; }

// Two consecutive RGB intervals at a shifted row position yf (even), or two
// empty intervals outside [0, S): a clamped address and a select.
template <typename TS>
__device__ __forceinline__ void far_pair_rgb_sel(const TS *row, int yf, int S, float4 &a, float4 &b) {
    const bool in = (unsigned)yf < (unsigned)S;
    const int yc = in ? yf : 0;
    const float4 va = ld4(row + yc), vb = ld4(row + yc + 1);
    a = in ? va : empty_interval<float4>();
    b = in ? vb : empty_interval<float4>();
}

// One pair of rows (y, y+1) of the three R_n planes at probe column x, cone
// pair ii (cones 2 ii and 2 ii + 1).  As the one-channel merge down, every
// operand is loaded before any is used, and TOP (n + 1 = N) builds the doubled
// edges of T_N from T_{N-1} and reads R_N = 0.  Per channel, the arithmetic
// and its order are those of Eq. 14 (odd x) and Eq. 15-17 (even x).
template <typename TS, bool TOP>
__device__ __forceinline__ void merge_down_rgb_pair(const DownArgs &a, int q, int x, int ii, int y,
                                                    float2 res[3]) {
    const int N = a.N, S = 1 << N, n = a.n, m = n + 1;
    const size_t SS = (size_t)S * S;
    const size_t plane = (size_t)a.nq * SS;
    const int jb = (1 << m) - 1 + 2 * ii;
    const float A[2] = {c_cone[jb], c_cone[jb + 1]};
    float acc0[3] = {0.f, 0.f, 0.f}, acc1[3] = {0.f, 0.f, 0.f};
    if (x & 1) {
        // Eq. 14: directions ii + up of this column to probe c of level n+1.
        const TS *Tx = reinterpret_cast<const TS *>(a.Tn) + q * a.en + (size_t)x * ((1 << n) + 1) * S;
        const int c = (x + 1) >> 1;
        const int yr = y + 2 * ii - (1 << n);
        float4 t0[2], t1[2];
        float2 rf[2][3];
#pragma unroll
        for (int up = 0; up < 2; ++up) {
            t0[up] = ld4(Tx + (size_t)(ii + up) * S + y);
            t1[up] = ld4(Tx + (size_t)(ii + up) * S + y + 1);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                rf[up][ch] = TOP ? make_float2(0.f, 0.f)
                                 : r_pair_sel(a.Rn1, (unsigned)(ch * plane + q * SS), N, m, c, 2 * ii + up,
                                              yr + 2 * up, 0.f);
        }
#pragma unroll
        for (int up = 0; up < 2; ++up) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                acc0[ch] += fmaf(t0[up].w, rf[up][ch].x, A[up] * chan(t0[up], ch));
                acc1[ch] += fmaf(t1[up].w, rf[up][ch].y, A[up] * chan(t1[up], ch));
            }
        }
    } else {
        // Eq. 15-17: probe c averaged with the doubled edge T_{n+1}(c, e2),
        // e2 = 2 ii + 2 up, to probe c + 1; at n = N-1 that edge is built here
        // as the merge up builds an even direction (Eq. 18).
        const int c = x >> 1;
        float4 t0[2], t1[2];
        if (TOP) {
            const TS *Tnear = reinterpret_cast<const TS *>(a.Tn) + q * a.en +
                              (size_t)(2 * c) * ((1 << n) + 1) * S;
            const TS *Tfar = Tnear + (size_t)((1 << n) + 1) * S;
            float4 n0[2], n1[2], f0[2], f1[2];
#pragma unroll
            for (int up = 0; up < 2; ++up) {
                n0[up] = ld4(Tnear + (size_t)(ii + up) * S + y);
                n1[up] = ld4(Tnear + (size_t)(ii + up) * S + y + 1);
                far_pair_rgb_sel(Tfar + (size_t)(ii + up) * S, y + 2 * ii + 2 * up - (1 << n), S,
                                 f0[up], f1[up]);
            }
#pragma unroll
            for (int up = 0; up < 2; ++up) {
                t0[up] = merge(n0[up], f0[up]);
                t1[up] = merge(n1[up], f1[up]);
            }
        } else {
            const TS *Tx = reinterpret_cast<const TS *>(a.Tn1) + q * a.en1 +
                           (size_t)c * ((1 << m) + 1) * S;
#pragma unroll
            for (int up = 0; up < 2; ++up) {
                t0[up] = ld4(Tx + (size_t)(2 * ii + 2 * up) * S + y);
                t1[up] = ld4(Tx + (size_t)(2 * ii + 2 * up) * S + y + 1);
            }
        }
        float2 ra[2][3], rb[2][3];
#pragma unroll
        for (int up = 0; up < 2; ++up) {
            const int yf = y + 4 * ii + 4 * up - (1 << m);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const unsigned rq = (unsigned)(ch * plane + q * SS);
                ra[up][ch] = TOP ? make_float2(0.f, 0.f)
                                 : r_pair_sel(a.Rn1, rq, N, m, c, 2 * ii + up, y, 0.f);
                rb[up][ch] = TOP ? make_float2(0.f, 0.f)
                                 : r_pair_sel(a.Rn1, rq, N, m, c + 1, 2 * ii + up, yf, 0.f);
            }
        }
#pragma unroll
        for (int up = 0; up < 2; ++up) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                acc0[ch] += 0.5f * (ra[up][ch].x + fmaf(t0[up].w, rb[up][ch].x, A[up] * chan(t0[up], ch)));
                acc1[ch] += 0.5f * (ra[up][ch].y + fmaf(t1[up].w, rb[up][ch].y, A[up] * chan(t1[up], ch)));
            }
        }
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) res[ch] = make_float2(acc0[ch], acc1[ch]);
}

// Merge down (Eq. 14-17) of RGB intervals into three planes, n >= 1, two
// consecutive y per thread.
template <typename TS>
__device__ void body_merge_down_rgb(const DownArgs &a, unsigned tile, int U, int tid) {
    const int N = a.N, S = 1 << N, n = a.n;
    const size_t SS = (size_t)S * S;
    const size_t plane = (size_t)a.nq * SS;
    const size_t total = (size_t)a.nq * (SS / 2);
    for (int uu = 0; uu < U; ++uu) {
        const size_t idx = ((size_t)tile * U + uu) * 256 + tid;
        if (idx >= total) return;
        const int y = (int)(idx & (S / 2 - 1)) * 2;
        const unsigned row = (unsigned)(idx >> (N - 1));
        const int q = row >> N;
        const unsigned r = row & (S - 1);
        const int x = r >> n, ii = r & ((1 << n) - 1);
        float2 res[3];
        if (n + 1 == N)
            merge_down_rgb_pair<TS, true>(a, q, x, ii, y, res);
        else
            merge_down_rgb_pair<TS, false>(a, q, x, ii, y, res);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
            *reinterpret_cast<float2 *>(a.R + ch * plane + q * SS + (size_t)r * S + y) = res[ch];
    }
}

// Tail of the RGB forward: levels 1 and 0 of the merge down, the gather and
// the sum of the four quadrants, as the one-channel tail, per channel.
template <int TILE> struct TailTileRgb {
    using T1 = TailTile<TILE>;
    static constexpr int plane = T1::plane;
    static constexpr int iv_bytes = 2 * plane * 16;
    static constexpr int r1_plane = T1::r1cols * 2 * T1::r1rows;  // floats per channel
    static constexpr int acc_plane = TILE * T1::acc_pitch;       // floats per channel
    static constexpr int lds = iv_bytes + 3 * r1_plane * 4 + 3 * acc_plane * 4;
};

__device__ __forceinline__ float r2_at3(const float *R2, int ro, int jj, int y, int S, bool cin) {
    const bool in = cin && (unsigned)y < (unsigned)S;
    const float v = R2[in ? (unsigned)(ro + jj * S + y) : 0u];
    return in ? v : 0.f;
}

template <int TILE>
__device__ void body_tail_rgb(const TailArgs &a, unsigned tile, char *lds, int tid) {
    using G1 = TailTile<TILE>;
    using G = TailTileRgb<TILE>;
    constexpr int H = G1::halo, P = G1::pitch, RR = G1::r1rows, AP = G1::acc_pitch;
    constexpr int span2 = G1::span * G1::span;
    constexpr int R1P = G::r1_plane, ACP = G::acc_plane;
    float4 *iv = reinterpret_cast<float4 *>(lds);
    float *r1 = reinterpret_cast<float *>(lds + G::iv_bytes);
    float *acc = reinterpret_cast<float *>(lds + G::iv_bytes + 3 * R1P * 4);
    const int N = a.N, S = 1 << N;
    const size_t SS = (size_t)S * S;
    const int tiles = (S + TILE - 1) / TILE;
    const int r0 = (int)(tile / tiles) * TILE, c0 = (int)(tile % tiles) * TILE;
    for (int i = tid; i < span2; i += 256) {
        const int lr = i / G1::span, lc = i % G1::span;
        const int r = r0 - H + lr, c = c0 - H + lc;
        const bool in = (unsigned)r < (unsigned)S && (unsigned)c < (unsigned)S;
        const size_t off = in ? (size_t)r * S + c : 0;
        const float e0 = in ? a.eps[off] : 0.f, e1 = in ? a.eps[SS + off] : 0.f;
        const float e2 = in ? a.eps[2 * SS + off] : 0.f, g = in ? a.sig[off] : 0.f;
        iv[lr * P + lc] = cell_interval_rgb(e0, e1, e2, g, 0.5f);
        iv[G::plane + lr * P + lc] = cell_interval_rgb(e0, e1, e2, g, kH2);
    }
    for (int i = tid; i < 3 * ACP; i += 256) acc[i] = 0.f;
    const size_t R2plane = (size_t)a.nq * SS;
    for (int g = 0; g < a.nq; ++g) {
        const int q = a.q0 + g;
        const float *R2 = a.R2 + (size_t)g * SS;
        const int u_lo = q == 0 ? c0 : q == 1 ? S - TILE - c0 : q == 2 ? r0 : S - TILE - r0;
        const int w_lo = q < 2 ? r0 : c0;
        const int su = q == 0 ? 1 : q == 1 ? -1 : q == 2 ? P : -P;
        const int sw = q < 2 ? P : 1;
        const int base = q == 1 ? H * P + TILE - 1 + H : q == 3 ? (TILE - 1 + H) * P + H : H * P + H;
        const int c1_lo = u_lo / 2 + 1;
        const int cmax = S >> 2;
        __syncthreads();
        // R_1 at odd level-1 columns (Eq. 14 at level 1)
        constexpr int n_odd = (TILE / 4 + 1) * RR;
        for (int i = tid; i < n_odd; i += 256) {
            const int j = 2 * (i / RR), wl = i % RR;
            const int cp = c1_lo + j, w = w_lo - 2 + wl;
            float v0[3] = {0.f, 0.f, 0.f}, v1[3] = {0.f, 0.f, 0.f};
            if (cp >= 0 && cp < (S >> 1) && (unsigned)w < (unsigned)S) {
                const float4 *ivp = iv + base + (2 * cp - u_lo) * su + (w - w_lo) * sw;
                const float4 t0 = tail_ray<2, 4, G::plane>(ivp, su, sw);
                const float4 t1 = tail_ray<3, 4, G::plane>(ivp, su, sw);
                const float4 t2 = tail_ray<4, 4, G::plane>(ivp, su, sw);
                const int c = (cp + 1) >> 1;
                const bool cin = c < cmax;
                const int ro = (cin ? c : 0) * 4 * S;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float *R2c = R2 + ch * R2plane;
                    v0[ch] = fmaf(t0.w, r2_at3(R2c, ro, 0, w - 2, S, cin), c_cone[3] * chan(t0, ch)) +
                             fmaf(t1.w, r2_at3(R2c, ro, 1, w, S, cin), c_cone[4] * chan(t1, ch));
                    v1[ch] = fmaf(t1.w, r2_at3(R2c, ro, 2, w, S, cin), c_cone[5] * chan(t1, ch)) +
                             fmaf(t2.w, r2_at3(R2c, ro, 3, w + 2, S, cin), c_cone[6] * chan(t2, ch));
                }
            }
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                r1[ch * R1P + (2 * j) * RR + wl] = v0[ch];
                r1[ch * R1P + (2 * j + 1) * RR + wl] = v1[ch];
            }
        }
        // R_1 at even level-1 columns (Eq. 15-17 at level 1)
        constexpr int n_even = (TILE / 4) * RR;
        for (int i = tid; i < n_even; i += 256) {
            const int j = 2 * (i / RR) + 1, wl = i % RR;
            const int cp = c1_lo + j, w = w_lo - 2 + wl;
            float v0[3] = {0.f, 0.f, 0.f}, v1[3] = {0.f, 0.f, 0.f};
            if (cp >= 0 && cp < (S >> 1) && (unsigned)w < (unsigned)S) {
                const float4 *ivp = iv + base + (2 * cp - u_lo) * su + (w - w_lo) * sw;
                const float4 t0 = tail_ray<5, 8, G::plane>(ivp, su, sw);
                const float4 t2 = tail_ray<7, 8, G::plane>(ivp, su, sw);
                const float4 t4 = tail_ray<9, 8, G::plane>(ivp, su, sw);
                const int c = cp >> 1;
                const bool cin = c + 1 < cmax;
                const int ro = c * 4 * S, ro1 = (cin ? c + 1 : 0) * 4 * S;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float *R2c = R2 + ch * R2plane;
                    v0[ch] = 0.5f * (r2_at3(R2c, ro, 0, w, S, true) +
                                     fmaf(t0.w, r2_at3(R2c, ro1, 0, w - 4, S, cin), c_cone[3] * chan(t0, ch))) +
                             0.5f * (r2_at3(R2c, ro, 1, w, S, true) +
                                     fmaf(t2.w, r2_at3(R2c, ro1, 1, w, S, cin), c_cone[4] * chan(t2, ch)));
                    v1[ch] = 0.5f * (r2_at3(R2c, ro, 2, w, S, true) +
                                     fmaf(t2.w, r2_at3(R2c, ro1, 2, w, S, cin), c_cone[5] * chan(t2, ch))) +
                             0.5f * (r2_at3(R2c, ro, 3, w, S, true) +
                                     fmaf(t4.w, r2_at3(R2c, ro1, 3, w + 4, S, cin), c_cone[6] * chan(t4, ch)));
                }
            }
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                r1[ch * R1P + (2 * j) * RR + wl] = v0[ch];
                r1[ch * R1P + (2 * j + 1) * RR + wl] = v1[ch];
            }
        }
        __syncthreads();
        // R_0 at x = u + 1 for every pixel (u, w) of the tile, added to the sums
        constexpr int SP = 256 / TILE, IT = TILE * TILE / 256;
        const int wl = tid % TILE, w = w_lo + wl, slot0 = tid / TILE;
        const int au = q == 0 ? 1 : q == 1 ? -1 : q == 2 ? AP : -AP;
        const int aw = q < 2 ? AP : 1;
        const int abase = q == 1 ? TILE - 1 : q == 3 ? (TILE - 1) * AP : 0;
        const float4 *ivw = iv + base + su + wl * sw;
        float *accw = acc + abase + wl * aw;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int ul;
            if constexpr (IT >= 2)
                ul = 2 * (slot0 + SP * (it % (IT / 2))) + (it >= IT / 2 ? 1 : 0);
            else
                ul = slot0 < SP / 2 ? 2 * slot0 : 2 * (slot0 - SP / 2) + 1;
            const int u = u_lo + ul;
            if (u < 0 || u >= S || w >= S) continue;
            const float4 *ivp = ivw + ul * su;
            float v[3] = {0.f, 0.f, 0.f};
            if ((ul & 1) == 0) {
                const float4 t0 = tail_ray<0, 2, G::plane>(ivp, su, sw);
                const float4 t1 = tail_ray<1, 2, G::plane>(ivp, su, sw);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float *rj = r1 + ch * R1P + ul * RR + wl;
                    v[ch] = fmaf(t0.w, rj[1], c_cone[1] * chan(t0, ch)) +
                            fmaf(t1.w, rj[RR + 3], c_cone[2] * chan(t1, ch));
                }
            } else if (u + 1 < S) {
                const float4 t0 = tail_ray<2, 4, G::plane>(ivp, su, sw);
                const float4 t2 = tail_ray<4, 4, G::plane>(ivp, su, sw);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float *rj = r1 + ch * R1P + (ul - 1) * RR + wl;
                    v[ch] = 0.5f * (rj[2] + fmaf(t0.w, rj[2 * RR], c_cone[1] * chan(t0, ch))) +
                            0.5f * (rj[RR + 2] + fmaf(t2.w, rj[3 * RR + 4], c_cone[2] * chan(t2, ch)));
                }
            }
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) accw[ch * ACP + ul * au] += v[ch];
        }
    }
    __syncthreads();
    for (int i = tid; i < TILE * TILE; i += 256) {
        const int rl = i / TILE, cl = i % TILE;
        const int r = r0 + rl, c = c0 + cl;
        if (r < S && c < S) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) a.out[ch * SS + (size_t)r * S + c] = acc[ch * ACP + rl * AP + cl];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Reverse of the RGB solve.  The adjoint of an RGB interval is one float4
// (dL_r, dL_g, dL_b, dT) and an adjoint cascade level is three planes, as in
// the forward.  The merge's transpose keeps the channels apart in its radiance
// terms and gathers them in its transmittance term: for L_c = L_n,c + T_n L_f,c
// and T = T_n T_f, dL_n,c = dL_c, dL_f,c = dL_c T_n, dT_f = dT T_n and
// dT_n = sum_c dL_c L_f,c + dT T_f.  The radiance adjoints never depend on the
// transmittance adjoints, so each channel's radiance adjoints and d emission
// follow the one-channel reverse's arithmetic in its order (bitwise its
// result); only the transmittance adjoints and d sigma gather the channels,
// computing, storing and reading the medium's part once for all three.
// ---------------------------------------------------------------------------

// Adjoint of the merge down over three channel planes, transmittances shared
// (gather form, as body_merge_down_adj).
template <typename TS>
__device__ void body_merge_down_adj_rgb(const DownAdjArgs &a, unsigned tile, int U, int tid) {
    const int N = a.N, S = 1 << N, n = a.n, m = n + 1;
    const size_t SS = (size_t)S * S, plane = 4 * SS;
    for (int uu = 0; uu < U; ++uu) {
        const size_t idx = ((size_t)tile * U + uu) * 256 + tid;
        if (idx >= 2 * SS) return;
        const int yp = (int)(idx & (S / 2 - 1)) * 2;
        const unsigned row = (unsigned)(idx >> (N - 1));
        const int q = row >> N;
        const unsigned r = row & (S - 1);
        const int c = r >> m, jj = r & ((1 << m) - 1);
        const int ii = jj >> 1, up = jj & 1;
        const float *dRq = a.dR + q * SS;
        float2 f0[3], g[3], g2[3];
        float2 t = make_float2(0.f, 0.f), t2 = make_float2(0.f, 0.f);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            f0[ch] = *reinterpret_cast<const float2 *>(dRq + ch * plane +
                                                       ((size_t)(((2 * c) << n) | ii)) * S + yp);
            g[ch] = g2[ch] = make_float2(0.f, 0.f);
        }
        if (c >= 1) {
            // odd column 2c-1 (far end of Eq. 14) at row y = y' - (2e - 2^n)
            const int e = ii + up, x = 2 * c - 1;
            const int y = yp - (2 * e - (1 << n));  // odd when n = 0
            const size_t grow = ((size_t)((x << n) | ii)) * S;
            const TS *trow = reinterpret_cast<const TS *>(a.Tn) + q * a.en +
                             ((size_t)x * ((1 << n) + 1) + e) * S;
            if (n > 0) {
                const bool in = (unsigned)y < (unsigned)S;
                const int yc = in ? y : 0;
                const float4 ta = ld4(trow + yc), tb = ld4(trow + yc + 1);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float2 gv = *reinterpret_cast<const float2 *>(dRq + ch * plane + grow + yc);
                    g[ch] = in ? gv : make_float2(0.f, 0.f);
                }
                t = in ? make_float2(ta.w, tb.w) : make_float2(0.f, 0.f);
            } else {
                const bool in0 = (unsigned)y < (unsigned)S, in1 = (unsigned)(y + 1) < (unsigned)S;
                const int y0 = in0 ? y : 0, y1 = in1 ? y + 1 : 0;
                const float ta = ld4(trow + y0).w, tb = ld4(trow + y1).w;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float ga = dRq[ch * plane + grow + y0], gb = dRq[ch * plane + grow + y1];
                    g[ch] = make_float2(in0 ? ga : 0.f, in1 ? gb : 0.f);
                }
                t = make_float2(in0 ? ta : 0.f, in1 ? tb : 0.f);
            }
            // even column 2c-2 (far end of Eq. 17) at row y' - (2 e2 - 2^(n+1))
            const int e2 = 2 * ii + 2 * up, x2 = 2 * c - 2;
            const int y2 = yp - (2 * e2 - (1 << m));
            const bool in2 = (unsigned)y2 < (unsigned)S;
            const int y2c = in2 ? y2 : 0;
            const TS *t2row = reinterpret_cast<const TS *>(a.Tn1) + q * a.en1 +
                              ((size_t)(c - 1) * ((1 << m) + 1) + e2) * S;
            const float4 t2a = ld4(t2row + y2c), t2b = ld4(t2row + y2c + 1);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float2 gv = *reinterpret_cast<const float2 *>(
                    dRq + ch * plane + ((size_t)((x2 << n) | ii)) * S + y2c);
                g2[ch] = in2 ? gv : make_float2(0.f, 0.f);
            }
            t2 = in2 ? make_float2(t2a.w, t2b.w) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc0 = 0.5f * f0[ch].x, acc1 = 0.5f * f0[ch].y;
            acc0 = fmaf(g[ch].x, t.x, acc0);
            acc1 = fmaf(g[ch].y, t.y, acc1);
            acc0 = fmaf(0.5f * g2[ch].x, t2.x, acc0);
            acc1 = fmaf(0.5f * g2[ch].y, t2.y, acc1);
            *reinterpret_cast<float2 *>(a.dRn1 + ch * plane + q * SS + (size_t)r * S + yp) =
                make_float2(acc0, acc1);
        }
    }
}

// Adjoint of the RGB interval pyramid (gather form, as body_dT): dT_n from the
// merge down at levels n and n-1 and from the merge up of T_{n+1}, two
// consecutive y per thread, every operand loaded before the terms are added.
template <typename TS>
__device__ void body_dT_rgb(const DTArgs &a, unsigned tile, int U, int tid) {
    const int N = a.N, S = 1 << N, n = a.n;
    const size_t SS = (size_t)S * S, plane = 4 * SS;
    const int dirs = (1 << n) + 1;
    const unsigned rpq = (unsigned)(S >> n) * dirs;
    const size_t total = (size_t)4 * rpq * (S / 2);
    for (int uu = 0; uu < U; ++uu) {
        const size_t idx = ((size_t)tile * U + uu) * 256 + tid;
        if (idx >= total) return;
        const int y = (int)(idx & (S / 2 - 1)) * 2;
        const unsigned row = (unsigned)(idx >> (N - 1));
        const int q = (row >= rpq) + (row >= 2 * rpq) + (row >= 3 * rpq);
        const unsigned r = row - (unsigned)q * rpq;
        const int x = (int)div_rows(r, (unsigned)dirs), k = (int)(r - (unsigned)x * dirs);
        // (a) merge down at level n, odd x (Eq. 14)
        float2 ag[2][3], ar[2][3];
        float aA[2] = {0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) ag[i][ch] = ar[i][ch] = make_float2(0.f, 0.f);
        if (n < N && (x & 1)) {
            const int c = (x + 1) >> 1, yf = y + 2 * k - (1 << n);
            const bool rin = n + 1 < N && c < (S >> (n + 1));
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int ii = k - 1 + i, jj = 2 * k - 1 + i;
                if (ii < 0 || ii >= (1 << n)) continue;
                aA[i] = c_cone[(1 << (n + 1)) - 1 + jj];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    ag[i][ch] = *reinterpret_cast<const float2 *>(
                        a.dRn + ((unsigned)(ch * plane + q * SS) + ((unsigned)((x << n) | ii) << N) +
                                 (unsigned)y));
                    ar[i][ch] = ld2_r_at(rin, a.Rn1,
                                         (unsigned)(ch * plane + q * SS) +
                                             ((unsigned)((c << (n + 1)) | jj) << N),
                                      yf, S, n > 0, 0.f);
                }
            }
        }
        // (b) merge down at level n-1, even column 2x (Eq. 17)
        float2 bg[2][3], br[2][3];
        float bA[2] = {0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) bg[i][ch] = br[i][ch] = make_float2(0.f, 0.f);
        if (n >= 1 && (k & 1) == 0) {
            const int nm = n - 1, yf = y + 2 * k - (1 << n), xm = 2 * x;
            const bool rin = n < N && x + 1 < (S >> n);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int jj = k - 1 + i;
                if (jj < 0 || jj >= (1 << n)) continue;
                bA[i] = c_cone[(1 << n) - 1 + jj];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    bg[i][ch] = *reinterpret_cast<const float2 *>(
                        a.dRm + ((unsigned)(ch * plane + q * SS) +
                                 ((unsigned)((xm << nm) | (k / 2 - 1 + i)) << N) + (unsigned)y));
                    br[i][ch] = ld2_r_at(rin, a.Rn,
                                         (unsigned)(ch * plane + q * SS) +
                                             ((unsigned)(((x + 1) << n) | jj) << N),
                                      yf, S, true, 0.f);
                }
            }
        }
        // (c) merge up of T_{n+1} from T_n (Eq. 18-20, n >= 2: even shifts)
        float4 cg[3][2], cf[3][2];
        float cw[3] = {0.f, 0.f, 0.f};
        const bool near_role = (x & 1) == 0;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            cg[v][0] = cg[v][1] = make_float4(0.f, 0.f, 0.f, 0.f);
            cf[v][0] = cf[v][1] = empty_interval<float4>();
        }
        if (a.has_up) {
            const int H = 1 << n, odirs = 2 * H + 1;
            // 32-bit element offsets (a level holds fewer than 2^28 entries)
            const float4 *g0 = reinterpret_cast<const float4 *>(a.dTn1) +
                               ((unsigned)q * (unsigned)a.en1 + ((unsigned)((x >> 1) * odirs) << N));
            const TS *part = reinterpret_cast<const TS *>(a.Tn) +
                             ((unsigned)q * (unsigned)a.en + ((unsigned)((near_role ? x + 1 : x - 1) * dirs) << N));
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const int ko = v == 0 ? 2 * k : (v == 1 ? 2 * k + 1 : 2 * k - 1);
                const int kp = v == 0 ? k : (v == 1 ? k + 1 : k - 1);
                if (ko < 0 || ko > 2 * H) continue;
                cw[v] = v == 0 ? 1.f : 0.5f;
                if (near_role) {
                    far_pair_rgb(part + (size_t)kp * S, y + 2 * k - H, S, cf[v][0], cf[v][1]);
                    cg[v][0] = g0[(size_t)ko * S + y];
                    cg[v][1] = g0[(size_t)ko * S + y + 1];
                } else {
                    const int yo = y - (2 * kp - H);
                    const bool in = (unsigned)yo < (unsigned)S;
                    const int yc = in ? yo : 0;
                    const float4 t0 = ld4(part + (size_t)kp * S + yc), t1 = ld4(part + (size_t)kp * S + yc + 1);
                    const float4 h0 = g0[(size_t)ko * S + yc], h1 = g0[(size_t)ko * S + yc + 1];
                    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                    cf[v][0] = in ? t0 : z;
                    cf[v][1] = in ? t1 : z;
                    cg[v][0] = in ? h0 : z;
                    cg[v][1] = in ? h1 : z;
                }
            }
        }
        float gl[3][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
        float gt[2] = {0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                gl[ch][0] = fmaf(ag[i][ch].x, aA[i], gl[ch][0]);
                gl[ch][1] = fmaf(ag[i][ch].y, aA[i], gl[ch][1]);
                gt[0] = fmaf(ag[i][ch].x, ar[i][ch].x, gt[0]);
                gt[1] = fmaf(ag[i][ch].y, ar[i][ch].y, gt[1]);
            }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float g0x = 0.5f * bg[i][ch].x, g0y = 0.5f * bg[i][ch].y;
                gl[ch][0] = fmaf(g0x, bA[i], gl[ch][0]);
                gl[ch][1] = fmaf(g0y, bA[i], gl[ch][1]);
                gt[0] = fmaf(g0x, br[i][ch].x, gt[0]);
                gt[1] = fmaf(g0y, br[i][ch].y, gt[1]);
            }
        if (near_role) {
#pragma unroll
            for (int v = 0; v < 3; ++v)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const float4 g = cg[v][j], f = cf[v][j];
                    gl[0][j] = fmaf(cw[v], g.x, gl[0][j]);
                    gl[1][j] = fmaf(cw[v], g.y, gl[1][j]);
                    gl[2][j] = fmaf(cw[v], g.z, gl[2][j]);
                    gt[j] = fmaf(cw[v], fmaf(g.x, f.x, fmaf(g.y, f.y, fmaf(g.z, f.z, g.w * f.w))), gt[j]);
                }
        } else {
#pragma unroll
            for (int v = 0; v < 3; ++v)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const float4 g = cg[v][j], tn = cf[v][j];
                    gl[0][j] = fmaf(cw[v] * g.x, tn.w, gl[0][j]);
                    gl[1][j] = fmaf(cw[v] * g.y, tn.w, gl[1][j]);
                    gl[2][j] = fmaf(cw[v] * g.z, tn.w, gl[2][j]);
                    gt[j] = fmaf(cw[v] * g.w, tn.w, gt[j]);
                }
        }
        float4 *out = reinterpret_cast<float4 *>(a.dT) + q * a.en + (size_t)r * S + y;
        out[0] = make_float4(gl[0][0], gl[1][0], gl[2][0], gt[0]);
        out[1] = make_float4(gl[0][1], gl[1][1], gl[2][1], gt[1]);
    }
}

// Adjoint of the RGB traced levels (as body_seed_adj): each pixel sums, per
// half length, dLoss/dL_j of every channel and dLoss/dT_j over the pieces of
// every ray that cross it, then applies its cell derivatives once.
constexpr int kSeedAdjRgbLds = 3 * kAdjSpan * kAdjPitch * 16;
static_assert(12 * kAccPlane * 4 <= kSeedAdjRgbLds, "partial sums fit over the interval tile");

struct AdjSumsRgb {
    float dl[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};  // [half length][channel]
    float dt[3] = {0.f, 0.f, 0.f};
    template <int L>
    __device__ __forceinline__ void add(float d0, float d1, float d2, float t) {
        dl[L][0] += d0;
        dl[L][1] += d1;
        dl[L][2] += d2;
        dt[L] += t;
    }
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t dT_resource_rgb(const float2 *p, size_t entries) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2 *>(p), (short)0,
                                             (int)(entries * sizeof(float4)), (int)kBufferWord3);
}

template <int Q, int n, int rho, int k>
__device__ __forceinline__ void seed_adj_dir_rgb(__amdgpu_buffer_rsrc_t dTq, int S, int un, int w,
                                                 int lane_off, const float4 *ivp, AdjSumsRgb &sum) {
    constexpr int dirs = (1 << n) + 1, pieces = 2 << n;
    constexpr int L = piece_len(n, k);
    constexpr int plane = kAdjSpan * kAdjPitch;
    float4 g[2];
#pragma unroll
    for (int which = 0; which < 2; ++which) {
        const int j = adj_piece(n, rho, which);
        const int cj = (piece_du(j) - (rho & ((1 << n) - 1))) >> n;
        const int dwj = piece_dw(n, k, j);
        const int pw = w - dwj;
        const bool ok = un >= cj && (unsigned)pw < (unsigned)S;
        const unsigned off =
            ok ? (unsigned)(lane_off + ((k - cj * dirs) * S - dwj) * (int)sizeof(float4)) : kOutside;
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(dTq, off, 0, 0);
        g[which] = make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                               __uint_as_float(v[3]));
    }
#pragma unroll
    for (int which = 0; which < 2; ++which) {
        const int j = adj_piece(n, rho, which);
        float pre = 1.f;
        float4 suf = empty_interval<float4>();
#pragma unroll
        for (int i = pieces - 1; i >= 0; --i) {
            if (i == j) continue;
            const float4 c = ivp[L * plane + adj_lds_off<Q>(piece_du(i) - piece_du(j),
                                                             piece_dw(n, k, i) - piece_dw(n, k, j))];
            if (i > j) suf = merge(c, suf);
            else pre *= c.w;
        }
        const float4 gg = g[which];
        sum.add<L>(gg.x * pre, gg.y * pre, gg.z * pre,
                   pre * fmaf(gg.x, suf.x, fmaf(gg.y, suf.y, fmaf(gg.z, suf.z, gg.w * suf.w))));
    }
}

template <int Q, int n, int rho>
__device__ __forceinline__ void seed_adj_level_rgb(__amdgpu_buffer_rsrc_t dTq, int S, int u, int w,
                                                   const float4 *ivp, AdjSumsRgb &sum) {
    constexpr int dirs = (1 << n) + 1;
    const int un = u >> n;
    const int lane_off = (un * dirs * S + w) * (int)sizeof(float4);
    seed_adj_dir_rgb<Q, n, rho, 0>(dTq, S, un, w, lane_off, ivp, sum);
    seed_adj_dir_rgb<Q, n, rho, (1 << n)>(dTq, S, un, w, lane_off, ivp, sum);
    if constexpr (n >= 1) seed_adj_dir_rgb<Q, n, rho, (1 << n) / 2>(dTq, S, un, w, lane_off, ivp, sum);
    if constexpr (n == 2) {
        seed_adj_dir_rgb<Q, n, rho, 1>(dTq, S, un, w, lane_off, ivp, sum);
        seed_adj_dir_rgb<Q, n, rho, 3>(dTq, S, un, w, lane_off, ivp, sum);
    }
}

template <int Q, int rho>
__device__ __forceinline__ void seed_adj_levels_rgb(const SeedAdjArgs &a, int u, int w,
                                                    const float4 *ivp, AdjSumsRgb &sum) {
    const int S = 1 << a.N;
    // RGB levels hold 16-byte entries: quadrant Q starts Q e_n entries in
    seed_adj_level_rgb<Q, 0, 0>(dT_resource_rgb(a.dT0 + (size_t)Q * a.e0 * 2, a.e0), S, u, w, ivp, sum);
    seed_adj_level_rgb<Q, 1, rho & 1>(dT_resource_rgb(a.dT1 + (size_t)Q * a.e1 * 2, a.e1), S, u, w, ivp, sum);
    seed_adj_level_rgb<Q, 2, rho>(dT_resource_rgb(a.dT2 + (size_t)Q * a.e2 * 2, a.e2), S, u, w, ivp, sum);
}

template <int Q>
__device__ __forceinline__ void seed_adj_quadrant_rgb(const SeedAdjArgs &a, int v, int r, int c,
                                                      const float4 *ivp, AdjSumsRgb &sum) {
    const int S = 1 << a.N;
    const int u = Q == 0 ? c : Q == 1 ? S - 1 - c : Q == 2 ? r : S - 1 - r;
    const int w = Q < 2 ? r : c;
    switch ((Q == 0 || Q == 2) ? v : 3 - v) {
        case 0: seed_adj_levels_rgb<Q, 0>(a, u, w, ivp, sum); break;
        case 1: seed_adj_levels_rgb<Q, 1>(a, u, w, ivp, sum); break;
        case 2: seed_adj_levels_rgb<Q, 2>(a, u, w, ivp, sum); break;
        default: seed_adj_levels_rgb<Q, 3>(a, u, w, ivp, sum); break;
    }
}

__device__ __forceinline__ void body_seed_adj_rgb(const SeedAdjArgs &a, unsigned tile, char *lds,
                                                  int tid) {
    constexpr int P = kAdjPitch, plane = kAdjSpan * kAdjPitch, H = kAdjHalo;
    float4 *iv = reinterpret_cast<float4 *>(lds);
    const int S = 1 << a.N;
    const size_t SS = (size_t)S * S;
    const int tiles = (S + kAdjTile - 1) / kAdjTile;
    const int r0 = (int)(tile / tiles) * kAdjTile, c0 = (int)(tile % tiles) * kAdjTile;
    for (int i = tid; i < kAdjSpan * kAdjSpan; i += 256) {
        const int lr = i / kAdjSpan, lc = i % kAdjSpan;
        const int r = r0 - H + lr, c = c0 - H + lc;
        float e0 = 0.f, e1 = 0.f, e2 = 0.f, g = 0.f;
        if (r >= 0 && r < S && c >= 0 && c < S) {
            const size_t o = (size_t)r * S + c;
            e0 = a.eps[o];
            e1 = a.eps[SS + o];
            e2 = a.eps[2 * SS + o];
            g = a.sig[o];
        }
        const int l = lr * P + lc;
        iv[l] = cell_interval_rgb(e0, e1, e2, g, 0.5f);
        iv[plane + l] = cell_interval_rgb(e0, e1, e2, g, kH2);
        iv[2 * plane + l] = cell_interval_rgb(e0, e1, e2, g, kQ5);
    }
    __syncthreads();
    const int v = tid >> 6, lane = tid & 63;
    const int i4 = v + 4 * (lane >> 4), i16 = lane & 15;
    AdjSumsRgb sa;
    if (r0 + i16 < S && c0 + i4 < S) {
        const float4 *ivp = iv + i16 * P + i4;
        seed_adj_quadrant_rgb<0>(a, v, r0 + i16, c0 + i4, ivp, sa);
        seed_adj_quadrant_rgb<1>(a, v, r0 + i16, c0 + i4, ivp, sa);
    }
    const int r = r0 + i4, c = c0 + i16;
    const bool in = r < S && c < S;
    AdjSumsRgb sb;
    if (in) {
        const float4 *ivp = iv + i4 * P + i16;
        seed_adj_quadrant_rgb<2>(a, v, r, c, ivp, sb);
        seed_adj_quadrant_rgb<3>(a, v, r, c, ivp, sb);
    }
    __syncthreads();
    float *x = reinterpret_cast<float *>(lds);  // [12][16][kAccPitch]
    const int la = i16 * kAccPitch + i4;
#pragma unroll
    for (int L = 0; L < 3; ++L) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) x[(L * 3 + ch) * kAccPlane + la] = sa.dl[L][ch];
        x[(9 + L) * kAccPlane + la] = sa.dt[L];
    }
    __syncthreads();
    if (in) {
        const int lb = i4 * kAccPitch + i16;
        float dl[3][3], dt[3];
#pragma unroll
        for (int L = 0; L < 3; ++L) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) dl[L][ch] = x[(L * 3 + ch) * kAccPlane + lb] + sb.dl[L][ch];
            dt[L] = x[(9 + L) * kAccPlane + lb] + sb.dt[L];
        }
        const size_t o = (size_t)r * S + c;
        const float s = a.sig[o];
        float ds = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const CellDer d(a.eps[ch * SS + o], s);
            a.dE[ch * SS + o] = fmaf(dl[2][ch], d.le2, fmaf(dl[1][ch], d.le1, dl[0][ch] * d.le0));
            if (ch == 0) ds = fmaf(dt[2], d.ts2, fmaf(dt[1], d.ts1, dt[0] * d.ts0));
            ds = fmaf(dl[2][ch], d.ls2, fmaf(dl[1][ch], d.ls1, fmaf(dl[0][ch], d.ls0, ds)));
        }
        a.dS[o] = ds;
    }
    __syncthreads();
}

// The persistent kernel's one LDS buffer: the largest body it runs (the traced
// levels and the tail run there on 16x16 tiles).
constexpr int kMaxLds2 = kSeedAdjLds > SeedTile<16>::lds ? kSeedAdjLds : SeedTile<16>::lds;
constexpr int kMaxLds = kMaxLds2 > TailTile<16>::lds ? kMaxLds2 : TailTile<16>::lds;

// One tile of the persistent kernel.  The thread index reaches the body as a
// value the compiler cannot see through, created afresh for every tile: were
// it threadIdx.x itself, the values every inlined body derives from it would
// be hoisted out of the persistent loop and stay live across all of the other
// bodies (125 instead of 87 VGPRs; 212 instead of 44 bytes of spills in the
// 64-VGPR variant).  Its range is restated so that index arithmetic stays
// 32-bit.
__device__ __forceinline__ void run_phase(const Phase &p, unsigned tile, char *lds) {
    unsigned t = threadIdx.x & 255u;
    asm volatile("" : "+v"(t));
    __builtin_assume(t < 256u);
    const int tid = (int)t;
    switch (p.kind) {
        case PH_SEED: body_seed<16, float2>(p.a.seed, tile, lds, tid); break;  // planner sets tile 16
        case PH_UP: body_merge_up<float2>(p.a.up, tile, p.U, tid); break;
        case PH_DOWN: body_merge_down<float2>(p.a.down, tile, p.U, tid); break;
        case PH_TAIL: body_tail<16>(p.a.tail, tile, lds, tid); break;  // planner sets tile 16
        case PH_GATHER_ADJ: body_gather_adj(p.a.ga, tile, lds, tid); break;
        case PH_DOWN_ADJ: body_merge_down_adj<float2>(p.a.da, tile, p.U, tid); break;
        case PH_DT: body_dT<float2>(p.a.dt, tile, p.U, tid); break;
        case PH_SEED_ADJ: body_seed_adj(p.a.sa, tile, lds, tid); break;
        case PH_BLUR: body_blur(p.a.bl, tile, tid); break;
        case PH_BLUR_ADJ: body_blur_adj(p.a.bl, tile, tid); break;
        default: break;
    }
}

// ---------------------------------------------------------------------------
// Standalone kernels: one tile per block, one kernel per pass kind (so that
// profiles name the pass).
// ---------------------------------------------------------------------------

#define HRC_ELEMENTWISE_KERNEL(name, body, field)                                  \
    __global__ __launch_bounds__(256) void name(Phase p) {                         \
        body(p.a.field, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid()); \
    }
HRC_ELEMENTWISE_KERNEL(hrc_merge_up, body_merge_up<float2>, up)
HRC_ELEMENTWISE_KERNEL(hrc_merge_down, body_merge_down<float2>, down)
HRC_ELEMENTWISE_KERNEL(hrc_merge_up_f16, body_merge_up<half2_t>, up)
HRC_ELEMENTWISE_KERNEL(hrc_merge_down_f16, body_merge_down<half2_t>, down)
HRC_ELEMENTWISE_KERNEL(hrc_merge_down_adj, body_merge_down_adj<float2>, da)
HRC_ELEMENTWISE_KERNEL(hrc_interval_adj, body_dT<float2>, dt)
HRC_ELEMENTWISE_KERNEL(hrc_merge_down_adj_f16, body_merge_down_adj<half2_t>, da)
HRC_ELEMENTWISE_KERNEL(hrc_interval_adj_f16, body_dT<half2_t>, dt)
#undef HRC_ELEMENTWISE_KERNEL

__global__ __launch_bounds__(256) void hrc_seed(Phase p) {
    __shared__ __align__(16) char lds[SeedTile<32>::lds];
    body_seed<32, float2>(p.a.seed, xcd_tile(blockIdx.x, gridDim.x), lds, ltid());
}
__global__ __launch_bounds__(256) void hrc_seed_f16(Phase p) {
    __shared__ __align__(16) char lds[SeedTile<32>::lds];
    body_seed<32, half2_t>(p.a.seed, xcd_tile(blockIdx.x, gridDim.x), lds, ltid());
}
__global__ __launch_bounds__(256) void hrc_seed_adj(Phase p) {
    __shared__ __align__(16) char lds[kSeedAdjLds];
    body_seed_adj(p.a.sa, xcd_tile(blockIdx.x, gridDim.x), lds, ltid());
}
__global__ __launch_bounds__(256) void hrc_blur(Phase p) {
    body_blur(p.a.bl, xcd_tile(blockIdx.x, gridDim.x), ltid());
}
__global__ __launch_bounds__(256) void hrc_blur_adj(Phase p) {
    body_blur_adj(p.a.bl, xcd_tile(blockIdx.x, gridDim.x), ltid());
}
__global__ __launch_bounds__(256) void hrc_tail(Phase p) {
    __shared__ __align__(16) char lds[TailTile<32>::lds];
    body_tail<32>(p.a.tail, xcd_tile(blockIdx.x, gridDim.x), lds, ltid());
}
__global__ __launch_bounds__(256) void hrc_seed_rgb(Phase p) {
    __shared__ __align__(16) char lds[SeedTileRgb<16>::lds];
    body_seed_rgb<16, float4>(p.a.seed, xcd_tile(blockIdx.x, gridDim.x), lds, ltid());
}
__global__ __launch_bounds__(256) void hrc_seed_rgb_f16(Phase p) {
    __shared__ __align__(16) char lds[SeedTileRgb<16>::lds];
    body_seed_rgb<16, half4_t>(p.a.seed, xcd_tile(blockIdx.x, gridDim.x), lds, ltid());
}
__global__ __launch_bounds__(256) void hrc_merge_up_rgb(Phase p) {
    body_merge_up_rgb<float4>(p.a.up, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid());
}
__global__ __launch_bounds__(256) void hrc_merge_up_rgb_f16(Phase p) {
    body_merge_up_rgb<half4_t>(p.a.up, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid());
}
__global__ __launch_bounds__(256) void hrc_merge_down_rgb(Phase p) {
    body_merge_down_rgb<float4>(p.a.down, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid());
}
__global__ __launch_bounds__(256) void hrc_merge_down_rgb_f16(Phase p) {
    body_merge_down_rgb<half4_t>(p.a.down, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid());
}
__global__ __launch_bounds__(256) void hrc_tail_rgb(Phase p) {
    __shared__ __align__(16) char lds[TailTileRgb<16>::lds];
    body_tail_rgb<16>(p.a.tail, xcd_tile(blockIdx.x, gridDim.x), lds, ltid());
}
__global__ __launch_bounds__(256) void hrc_merge_down_adj_rgb(Phase p) {
    body_merge_down_adj_rgb<float4>(p.a.da, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid());
}
__global__ __launch_bounds__(256) void hrc_interval_adj_rgb(Phase p) {
    body_dT_rgb<float4>(p.a.dt, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid());
}
__global__ __launch_bounds__(256) void hrc_merge_down_adj_rgb_f16(Phase p) {
    body_merge_down_adj_rgb<half4_t>(p.a.da, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid());
}
__global__ __launch_bounds__(256) void hrc_interval_adj_rgb_f16(Phase p) {
    body_dT_rgb<half4_t>(p.a.dt, xcd_tile_blk(blockIdx.x, gridDim.x, p.xblk), p.U, ltid());
}
__global__ __launch_bounds__(256) void hrc_seed_adj_rgb(Phase p) {
    __shared__ __align__(16) char lds[kSeedAdjRgbLds];
    body_seed_adj_rgb(p.a.sa, xcd_tile(blockIdx.x, gridDim.x), lds, ltid());
}
__global__ __launch_bounds__(256) void hrc_gather_adj(Phase p) {
    __shared__ __align__(16) char lds[kGatherAdjLds];
    body_gather_adj(p.a.ga, blockIdx.x, lds, ltid());
}

// ---------------------------------------------------------------------------
// Persistent batch kernel.  Work items are groups of Q tiles of one phase
// (Q = 1 or 4 256-thread quarters per block), run side by side by the block's
// quarters (so every quarter passes the same barriers), in queues of steps: a queue's step t depends only on its
// steps before t.  Blocks claim chunks of consecutive items from their queue's
// counter and run them in order.  A block counts the items it finishes in the
// current step and publishes that count (one atomic add) when it reaches an
// item of a later step or runs out of items; before its first item of step t
// it waits until step t-1 of its queue is complete.  Thread 0 performs both
// for the block, between block barriers.  Publishing before waiting means no
// block ever waits while holding unpublished work, and every item of step t-1
// was claimed before any item of step t by a block that is running, so the
// queue always drains (no grid-wide co-residency is assumed).
//
// Visibility.  With one queue per XCD (xcd_local) every block of a queue runs
// on the XCD whose L2 holds what the queue's passes write (vector L1 caches
// write through to it): a publisher waits until its block's stores are
// complete, and a waiter invalidates its L1 after seeing the count, so the
// queue's scenes never write the L2 back mid-kernel.  With a single queue over
// all XCDs a publisher makes the block's stores visible to every XCD with one
// agent-scope release (an L2 write-back) per block and step.
// ---------------------------------------------------------------------------

constexpr unsigned kMaxSpins = 1u << 20;  // about a second of polling

// The XCD (accelerator complex die) this wave runs on.
__device__ __forceinline__ unsigned xcc_id() {
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 0xfu;
}

__device__ __forceinline__ unsigned *sched_line(unsigned *sched, unsigned line) {
    return sched + (size_t)line * kSchedStride;
}

template <int Q>
__device__ __forceinline__ void persistent_loop(const BatchTables &t, unsigned *sched, char *lds,
                                                unsigned &s_item) {
    // this quarter's LDS (the quarter is uniform over each wave)
    const unsigned quarter = Q == 1 ? 0u : __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);
    char *qlds = lds + quarter * kMaxLds;
    unsigned *error = sched_line(sched, kSchedError);
    const int q = t.xcd_local ? (int)xcc_id() : 0;
    if (q < t.nqueues) {
        unsigned *counter = sched_line(sched, kSchedClaim + q);
        unsigned *done = sched_line(sched, kSchedClaim + t.nqueues + t.q_step[q]);
        const unsigned *step_items = t.step_items + t.q_step[q];
        const int nsteps = t.q_step[q + 1] - t.q_step[q];
        const int seg_lo = t.q_seg[q], seg_hi = t.q_seg[q + 1];
        const unsigned total = t.q_items[q];
        int cur_step = -1;
        unsigned completed = 0;
        unsigned item = 0, claim_end = 0;  // this block's claimed items [item, claim_end)
        int seg = seg_lo;
        unsigned seg_end = 0;              // first item after segment seg
        for (;;) {
            if (item == claim_end) {
                // claim the next chunk (one thread), then make it a scalar for the block
                if (threadIdx.x == 0) s_item = atomicAdd(counter, t.chunk);
                __syncthreads();
                item = __builtin_amdgcn_readfirstlane(s_item);
                claim_end = item + t.chunk;
                __syncthreads();
            }
            int step = nsteps;
            if (item < total) {
                if (item >= seg_end || item < t.seg_start[seg]) {
                    int lo = seg_lo, hi = seg_hi - 1;  // last segment starting at or before the item
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (t.seg_start[mid] <= item) lo = mid;
                        else hi = mid - 1;
                    }
                    seg = __builtin_amdgcn_readfirstlane(lo);
                    seg_end = seg + 1 < seg_hi ? t.seg_start[seg + 1] : total;
                }
                step = __builtin_amdgcn_readfirstlane(t.seg_step[seg]);
            }
            if (step != cur_step) {
                if (cur_step >= 0) {
                    // publish this block's items of the step it is leaving
                    if (t.xcd_local) {
                        // every wave's stores have reached the XCD's L2 before
                        // the barrier, and so before thread 0's count (the
                        // memory clobber keeps the compiler from moving stores
                        // past the wait)
                        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                        __syncthreads();
                    } else {
                        // the block barrier orders every wave's stores before
                        // thread 0's agent-scope release, which then makes them
                        // visible to the other XCDs once for the whole block
                        __syncthreads();
                        if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    }
                    if (threadIdx.x == 0)
                        __hip_atomic_fetch_add(&done[(size_t)cur_step * kSchedStride], completed,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                cur_step = step;
                completed = 0;
                if (step >= nsteps) break;
                if (step > 0) {
                    if (threadIdx.x == 0) {
                        // Bounded wait on relaxed loads (an acquiring load would
                        // invalidate the caches on every poll); the acquire fence
                        // below orders the step's reads after the count is seen.
                        // A step that never completes (a planning bug, or the
                        // failure test's unreachable count) raises the error word
                        // and lets the queue drain instead of hanging.
                        const unsigned *cfg = sched_line(sched, kSchedConfig);
                        const unsigned limit = cfg[0] ? cfg[0] : kMaxSpins;
                        const unsigned need = step_items[step - 1] + cfg[1];
                        const unsigned *d = &done[(size_t)(step - 1) * kSchedStride];
                        unsigned spins = 0;
                        while (__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                               need) {
                            if (++spins > limit) {
                                __hip_atomic_fetch_or(error, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(2);
                        }
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                    __syncthreads();  // the other waves read after thread 0's acquire
                }
            }
            const int pi = __builtin_amdgcn_readfirstlane(t.seg_phase[seg]);
            const unsigned tile =
                __builtin_amdgcn_readfirstlane(item - t.seg_start[seg]) * Q + quarter;
            run_phase(t.phases[pi], tile, qlds);
            ++completed;
            ++item;
        }
    }
    // The last block to finish checks that every queue completed its last step
    // (a queue whose XCD ran no block of the grid would not have).
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned before = __hip_atomic_fetch_add(sched_line(sched, kSchedExit), 1u,
                                                       __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (before + 1 == gridDim.x) {
            for (int qq = 0; qq < t.nqueues; ++qq) {
                const int ns = t.q_step[qq + 1] - t.q_step[qq];
                if (ns == 0) continue;
                const int last = t.q_step[qq + 1] - 1;
                const unsigned got = __hip_atomic_load(
                    sched_line(sched, kSchedClaim + t.nqueues + last), __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_AGENT);
                if (got < t.step_items[last])
                    __hip_atomic_fetch_or(error, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// Two block sizes (four tiles side by side, or one) and two register budgets
// for the same loop: the full budget, or 64 VGPRs (eight waves per SIMD, at
// the cost of some spills in the larger bodies).  The batch planner times all
// four.
__global__ __launch_bounds__(1024) void hrc_persistent(const BatchTables t, unsigned *sched) {
    __shared__ __align__(16) char lds[4 * kMaxLds];
    __shared__ unsigned s_item;
    persistent_loop<4>(t, sched, lds, s_item);
}
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
void hrc_persistent_dense(const BatchTables t, unsigned *sched) {
    __shared__ __align__(16) char lds[4 * kMaxLds];
    __shared__ unsigned s_item;
    persistent_loop<4>(t, sched, lds, s_item);
}
__global__ __launch_bounds__(256) void hrc_persistent_1(const BatchTables t, unsigned *sched) {
    __shared__ __align__(16) char lds[kMaxLds];
    __shared__ unsigned s_item;
    persistent_loop<1>(t, sched, lds, s_item);
}
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
void hrc_persistent_1_dense(const BatchTables t, unsigned *sched) {
    __shared__ __align__(16) char lds[kMaxLds];
    __shared__ unsigned s_item;
    persistent_loop<1>(t, sched, lds, s_item);
}

typedef void (*PersistentKernel)(const BatchTables, unsigned *);
static PersistentKernel persistent_kernel(int variant) {
    switch (variant) {
        case 0: return hrc_persistent;
        case 1: return hrc_persistent_dense;
        case 2: return hrc_persistent_1;
        default: return hrc_persistent_1_dense;
    }
}

// Clears words [from, n) of the scheduler state (a kernel rather than a memset
// so that it can be captured in a graph and replayed).
__global__ void hrc_clear_u32(unsigned *p, unsigned from, unsigned n) {
    unsigned i = from + blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// The XCD of every block (thread 0 writes it), for the planner to map queues.
__global__ __launch_bounds__(1024) void hrc_xcd_probe(unsigned *out) {
    if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

// Sets *flag when any element of a or b is negative or not finite.
__global__ __launch_bounds__(256) void hrc_validate(const float *a, const float *b, size_t n,
                                                  int *flag) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t stride = (size_t)gridDim.x * 256;
    for (; i < n; i += stride) {
        float x = a[i], y = b[i];
        if (!(x >= 0.f && x <= 3.4e38f) || !(y >= 0.f && y <= 3.4e38f)) *flag = 1;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers and phase builders
// ---------------------------------------------------------------------------

unsigned phase_tiles(const Phase &p) {
    auto cdiv = [](size_t a, size_t b) { return (unsigned)((a + b - 1) / b); };
    const int N = [&] {
        switch (p.kind) {
            case PH_SEED: return p.a.seed.N;
            case PH_UP: return p.a.up.N;
            case PH_DOWN: return p.a.down.N;
            case PH_TAIL: return p.a.tail.N;
            case PH_GATHER_ADJ: return p.a.ga.N;
            case PH_DOWN_ADJ: return p.a.da.N;
            case PH_DT: return p.a.dt.N;
            case PH_SEED_ADJ: return p.a.sa.N;
            case PH_BLUR:
            case PH_BLUR_ADJ: return p.a.bl.N;
            case PH_SEED_RGB: return p.a.seed.N;
            case PH_UP_RGB: return p.a.up.N;
            case PH_DOWN_RGB: return p.a.down.N;
            case PH_TAIL_RGB: return p.a.tail.N;
            case PH_DOWN_ADJ_RGB: return p.a.da.N;
            case PH_DT_RGB: return p.a.dt.N;
            case PH_SEED_ADJ_RGB: return p.a.sa.N;
        }
        return 0;
    }();
    const size_t S = size_t(1) << N, SS = S * S;
    const unsigned t32 = (unsigned)((S + 31) / 32);
    const size_t per = (size_t)256 * (p.U > 0 ? p.U : 1);
    switch (p.kind) {
        case PH_TAIL: {
            const unsigned t = (unsigned)((S + p.a.tail.tile - 1) / p.a.tail.tile);
            return t * t;
        }
        case PH_GATHER_ADJ: return 4 * t32 * t32;
        case PH_SEED: {
            const unsigned t = (unsigned)((S + p.a.seed.tile - 1) / p.a.seed.tile);
            return t * t;
        }
        case PH_UP:  // pairs of y per thread: one, two with 16-bit intervals
            return cdiv((size_t)p.a.up.nq * t_level_entries(N, p.a.up.n) / (p.a.up.half ? 4 : 2), per);
        case PH_DT:  // two probe columns per thread at levels 0 and 1
            return cdiv(4 * t_level_entries(N, p.a.dt.n) / (p.a.dt.n <= 1 && p.a.dt.n < N ? 4 : 2), per);
        case PH_DT_RGB: return cdiv(4 * t_level_entries(N, p.a.dt.n) / 2, per);
        case PH_DOWN: return cdiv((size_t)p.a.down.nq * SS / (p.a.down.half ? 4 : 2), per);
        case PH_DOWN_ADJ:
        case PH_DOWN_ADJ_RGB: return cdiv(4 * SS / 2, per);
        case PH_BLUR:
        case PH_BLUR_ADJ:
        case PH_SEED_ADJ:
        case PH_SEED_ADJ_RGB:
        case PH_SEED_RGB:
        case PH_TAIL_RGB: {
            const unsigned t16 = (unsigned)((S + 15) / 16);
            return t16 * t16;
        }
        case PH_UP_RGB: return cdiv((size_t)p.a.up.nq * t_level_entries(N, p.a.up.n) / 2, per);
        case PH_DOWN_RGB: return cdiv((size_t)p.a.down.nq * SS / 2, per);
    }
    return 0;
}

hipError_t upload_cone_table(const float *host_table) {
    return hipMemcpyToSymbol(HIP_SYMBOL(c_cone), host_table, sizeof(float) * kConeTable);
}

hipError_t launch_phase(const Phase &p, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    unsigned tiles = phase_tiles(p);
    if (tiles == 0) return hipSuccess;
    void (*k)(Phase) = nullptr;
    switch (p.kind) {
        case PH_SEED: k = p.a.seed.half ? hrc_seed_f16 : hrc_seed; break;
        case PH_UP: k = p.a.up.half ? hrc_merge_up_f16 : hrc_merge_up; break;
        case PH_DOWN: k = p.a.down.half ? hrc_merge_down_f16 : hrc_merge_down; break;
        case PH_TAIL: k = hrc_tail; break;
        case PH_GATHER_ADJ: k = hrc_gather_adj; break;
        case PH_DOWN_ADJ: k = p.a.da.half ? hrc_merge_down_adj_f16 : hrc_merge_down_adj; break;
        case PH_DT: k = p.a.dt.half ? hrc_interval_adj_f16 : hrc_interval_adj; break;
        case PH_SEED_ADJ: k = hrc_seed_adj; break;
        case PH_BLUR: k = hrc_blur; break;
        case PH_BLUR_ADJ: k = hrc_blur_adj; break;
        case PH_SEED_RGB: k = p.a.seed.half ? hrc_seed_rgb_f16 : hrc_seed_rgb; break;
        case PH_UP_RGB: k = p.a.up.half ? hrc_merge_up_rgb_f16 : hrc_merge_up_rgb; break;
        case PH_DOWN_RGB: k = p.a.down.half ? hrc_merge_down_rgb_f16 : hrc_merge_down_rgb; break;
        case PH_TAIL_RGB: k = hrc_tail_rgb; break;
        case PH_DOWN_ADJ_RGB: k = p.a.da.half ? hrc_merge_down_adj_rgb_f16 : hrc_merge_down_adj_rgb; break;
        case PH_DT_RGB: k = p.a.dt.half ? hrc_interval_adj_rgb_f16 : hrc_interval_adj_rgb; break;
        case PH_SEED_ADJ_RGB: k = hrc_seed_adj_rgb; break;
        default: return hipErrorInvalidValue;
    }
    if (start || stop)
        hipExtLaunchKernelGGL(k, dim3(tiles), dim3(256), 0, s, start, stop, 0, p);
    else
        hipLaunchKernelGGL(k, dim3(tiles), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_persistent(const BatchTables &t, unsigned *sched, int grid, int variant,
                             hipStream_t s) {
    const unsigned from = kSchedExit * kSchedStride;
    const unsigned n = (unsigned)sched_words(t.nqueues, t.q_step[t.nqueues]);
    hipLaunchKernelGGL(hrc_clear_u32, dim3((n - from + 255) / 256), dim3(256), 0, s, sched, from,
                       n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(persistent_kernel(variant), dim3(grid),
                       dim3(256 * persistent_quarters(variant)), 0, s, t, sched);
    return hipGetLastError();
}

hipError_t launch_xcd_probe(unsigned *out, int grid, int variant, hipStream_t s) {
    hipLaunchKernelGGL(hrc_xcd_probe, dim3(grid), dim3(256 * persistent_quarters(variant)), 0, s,
                       out);
    return hipGetLastError();
}

hipError_t persistent_occupancy(int variant, int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks_per_cu, persistent_kernel(variant), 256 * persistent_quarters(variant), 0);
}

// Multiple bounces: the in-scattering source of the next bounce and the reverse
// step of that update (elementwise, grid-stride).
constexpr float kInvTwoPi = 0.15915494309189533577f;

__global__ __launch_bounds__(256) void hrc_scatter_source(const float *eps0, const float *sig,
                                                          const float *alb, const float *F,
                                                          float *out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        out[i] = eps0[i] + alb[i] * sig[i] * F[i] * kInvTwoPi;
}

__global__ __launch_bounds__(256) void hrc_scatter_adj(const float *dE, const float *dS,
                                                       const float *F_prev, const float *sig,
                                                       const float *alb, float *g, float *d_eps,
                                                       float *d_sig, float *d_alb, size_t n,
                                                       int assign) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (size_t)gridDim.x * 256) {
        const float de = dE[i];
        float ds = dS[i];
        float da = 0.f;
        if (F_prev) {
            const float fp = F_prev[i] * de * kInvTwoPi;
            ds += alb[i] * fp;
            da = sig[i] * fp;
            g[i] = alb[i] * sig[i] * de * kInvTwoPi;
        }
        d_eps[i] = assign ? de : d_eps[i] + de;
        d_sig[i] = assign ? ds : d_sig[i] + ds;
        if (F_prev) d_alb[i] = assign ? da : d_alb[i] + da;
        else if (assign) d_alb[i] = 0.f;  // one bounce: no albedo dependence
    }
}

static unsigned elementwise_blocks(size_t n) {
    size_t b = (n + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : b);
}

hipError_t launch_scatter_source(const float *eps0, const float *sig, const float *alb,
                                 const float *F, float *out, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(hrc_scatter_source, dim3(elementwise_blocks(n)), dim3(256), 0, s, eps0,
                       sig, alb, F, out, n);
    return hipGetLastError();
}

hipError_t launch_scatter_adj(const float *dE, const float *dS, const float *F_prev,
                              const float *sig, const float *alb, float *g, float *d_eps,
                              float *d_sig, float *d_alb, size_t n, int assign, hipStream_t s) {
    hipLaunchKernelGGL(hrc_scatter_adj, dim3(elementwise_blocks(n)), dim3(256), 0, s, dE, dS,
                       F_prev, sig, alb, g, d_eps, d_sig, d_alb, n, assign);
    return hipGetLastError();
}

hipError_t launch_validate(const float *a, const float *b, size_t n, int *flag,
                           hipStream_t s) {
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(hrc_validate, dim3(blocks), dim3(256), 0, s, a, b, n, flag);
    return hipGetLastError();
}

}  // namespace hrc
