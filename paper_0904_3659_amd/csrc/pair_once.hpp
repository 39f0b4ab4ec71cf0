// The pair-once block evaluation of Eq. (gravity) (Sec. I), shared by the
// single-system forward kernel (forward_sym.hip) and the batched ensemble
// kernel (batched.hip).
//
// Every unordered pair is computed once: the term of pair (i, j) gives
// m_j d r^3 to a_i and, by the antisymmetry of the softened force (one eps2
// for all pairs), -m_i d r^3 to a_j; the potential term gives m_j r to p_i
// and m_i r to p_j.  That shares the difference, distance, rsqrt and r^3 of
// both ordered pairs.
//
// Blocks and the ring
//   A system of n particles is cut into M blocks of P = W*64*K.  The caller
//   (one workgroup) owns block I, chunk c of C: it keeps block I in VGPRs
//   (K rows per lane, W waves) and meets
//     - its own block (the diagonal), pair-once between different 64-row
//       tiles and as ordered pairs (j == i removed by index) within a tile,
//       and
//     - the blocks J = I + delta (mod M) for delta = 1..H_I (the ring), with
//       H_I = (M-1)/2, plus delta = M/2 when M is even and I < M/2,
//   so every unordered pair of distinct blocks is met exactly once.  The
//   block's tile sequence (diagonal tiles, then ring tiles delta-major) is
//   shared evenly among the C chunks.
//
// j-tiles of 64 particles are staged in LDS twice over (entries e and
// e + 64 hold particle e).  On a ring tile, lane l at step s (0..63) meets
// particle (l + s) mod 64 of the tile, read from entry l + s: each step is a
// permutation of the 64 particles over the 64 lanes, and the entry index
// needs no wrap, so the unrolled loop addresses LDS with immediate offsets
// from one base.  The j-side sums live in 128 per-wave LDS slots in the same
// way: at step s lane l adds its K terms to slot l + s (read-modify-write),
// so particle e collects in slots e and e + 64.  No two lanes touch the
// same slot in a step; a slot's next writer is another lane of the same
// wave, and one wave's LDS accesses complete in issue order, so the sums are
// exact read-modify-writes in a fixed order (no atomics; LDS atomics
// serialise and were 4x slower).  After the 64 steps the W waves' slot
// pairs are added in wave order and written as the tile's partial.
//
// Ring groups and partials.  The ring offsets are processed in groups of
// consecutive deltas, one launch per group, so that library memory stays
// O((C + G) n) instead of O(n^2 / P): launch g covers deltas [d_lo, d_hi)
// (the first group also the diagonal, delta 0) and writes float4 partials
// [C + G][n]: slots 0..C-1 hold the i-side sums of the C chunks over the
// group's tiles, slot C + delta - max(d_lo, 1) holds what particle j in
// block J received from block J - delta.  A fold kernel then adds each
// particle's slots of the group, in fixed order and in float64, to its
// running sum (the last group's fold rounds it and stores a, p).  No
// atomics, no cross-workgroup races: the result is bitwise reproducible for
// a given variant, n, chunk count and group size.
//
// Padding: rows past n take position +1e18 and mass 0, tile slots past n
// take -1e18 and mass 0, so padded terms are exactly zero for finite
// positions below 1e17 in magnitude.
#pragma once

#include "common.hpp"

#include <cstdlib>

namespace nbody {

constexpr float kPadRow = 1e18f;
constexpr float kPadCol = -1e18f;

// LDS entries per staged j-tile (64 particles, stored twice) and per wave's
// j-side slots.
constexpr int kTileLds = 128;
constexpr int kSlotLds = 128;

__host__ __device__ __forceinline__ int ring_len(int I, int M)
{
    return (M - 1) / 2 + (((M & 1) == 0 && I < M / 2) ? 1 : 0);
}

// Number of j-side slots block J of an M-block system receives.
__host__ __device__ __forceinline__ int ring_in(int J, int M)
{
    return (M - 1) / 2 + (((M & 1) == 0 && J >= M / 2) ? 1 : 0);
}

// The deltas of group [d_lo, d_hi) that have a j-side slot (the diagonal,
// delta 0, has none): [max(d_lo, 1), d_hi).
__host__ __device__ __forceinline__ int group_first_delta(int d_lo) { return d_lo > 0 ? d_lo : 1; }

// Fold of one ring group: particle j (block J) adds its C chunk slots and
// the j-side slots of the group's deltas its block received, deltas
// [dj, min(d_hi, ring_in(J, M) + 1)), in slot order, each widened to
// float64.  Four groups of 64 threads each add a contiguous quarter of the
// slots, and the four group sums are added in group order; the group's sum
// is then added to the particle's running sum acc (FIRST: acc is not read;
// LAST: the result is rounded once and xyz goes to out3[j][3], w to out1[j],
// skipped when out1 is NULL, followed by the leap-frog update `e` with EPI).
// A fixed order throughout: bitwise reproducible.  A workgroup covers 64
// particles.  acc is [n] double4 and is neither read nor written when the
// fold is both FIRST and LAST.
template <int PB, bool EPI = false>
__global__ __launch_bounds__(256) void slot_fold_kernel(const float4 *__restrict__ partial, int n,
                                                        int M, int C, int d_lo, int d_hi,
                                                        int first, int last, double4 *acc,
                                                        float *out3, float *out1, LfEpi e)
{
    __shared__ double4 red[4][64];
    const int l = threadIdx.x & 63;
    const int g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + l;
    double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
    if (j < n) {
        const int dj = group_first_delta(d_lo);
        const int recv = min(d_hi, ring_in(j / PB, M) + 1) - dj;
        const int S = C + (recv > 0 ? recv : 0);
        const int q = (S + 3) / 4;
        const int k1 = min(S, (g + 1) * q);
#pragma unroll 4
        for (int k = g * q; k < k1; ++k) {
            const float4 v = partial[(size_t)k * n + j];
            s.x += (double)v.x;
            s.y += (double)v.y;
            s.z += (double)v.z;
            s.w += (double)v.w;
        }
    }
    red[g][l] = s;
    __syncthreads();
    if (g != 0 || j >= n) return;
    double4 t = red[0][l];
#pragma unroll
    for (int g2 = 1; g2 < 4; ++g2) {
        const double4 v = red[g2][l];
        t.x += v.x;
        t.y += v.y;
        t.z += v.z;
        t.w += v.w;
    }
    if (!first) {
        const double4 r = acc[j];
        t.x += r.x;
        t.y += r.y;
        t.z += r.z;
        t.w += r.w;
    }
    if (!last) {
        acc[j] = t;
        return;
    }
    const float4 f = make_float4((float)t.x, (float)t.y, (float)t.z, (float)t.w);
    if constexpr (EPI) {
        lf_finish(e, j, f, out3, out1);
    } else {
        out3[3 * j + 0] = f.x;
        out3[3 * j + 1] = f.y;
        out3[3 * j + 2] = f.z;
        if (out1) out1[j] = f.w;
    }
}

// Launch plan of a single-system pair-once evaluation: M blocks of P
// particles, C chunks per block, D = M/2 ring deltas processed in `groups`
// launches of G deltas each (the first also the diagonal).  Workspace:
// partials [C + G][n] float4 and, with more than one group, a float64
// running sum [n] double4.
struct SymPlan {
    int M = 0, C = 0, G = 0, groups = 0;
    size_t partial_bytes = 0, acc_bytes = 0;
    size_t bytes() const { return partial_bytes + acc_bytes; }
};

// Plan for n particles in blocks of P, given the number of workgroups the
// device holds at once (resident; the chunk count fills them, divided by
// occ) and a workspace budget in bytes.  Returns false if even one delta
// per group and one chunk per block exceed the budget.
inline bool sym_plan(int64_t n, int P, int64_t resident, int occ, size_t budget, SymPlan *out)
{
    SymPlan pl;
    const int TPB = P / 64;
    pl.M = (int)((n + P - 1) / P);
    const int D = pl.M / 2;  // ring deltas 1..D
    int64_t C = resident / ((int64_t)pl.M * occ);
    const int64_t max_c = (int64_t)(D + 1) * TPB;  // tiles of a block's sequence
    C = C < 1 ? 1 : (C > max_c ? max_c : C);
    const size_t slot = 16 * (size_t)n;          // one float4 per particle
    const int64_t slots = (int64_t)(budget / slot);
    if (C + D <= slots || D == 0) {
        pl.C = (int)C;
        pl.G = D;
        pl.groups = 1;
    } else {
        // several groups: room for C + G slots plus the running sum (two
        // slots' worth); the chunks take at most half of the slots
        if (slots < 4) return false;
        const int64_t half = (slots - 2) / 2;
        if (C > half) C = half;
        const int64_t gmax = slots - C - 2;
        pl.groups = (int)((D + gmax - 1) / gmax);
        pl.G = (D + pl.groups - 1) / pl.groups;
        const int64_t cg = (int64_t)pl.G * TPB;  // tiles per block in a later group
        pl.C = (int)(C > cg ? cg : C);
    }
    // the running sum starts on a 256-byte boundary (double4 needs 32)
    pl.partial_bytes = (slot * (size_t)(pl.C + pl.G) + 255) / 256 * 256;
    pl.acc_bytes = pl.groups > 1 ? 32 * (size_t)n : 0;
    *out = pl;
    return true;
}

// Ring deltas [d_lo, d_hi) of group g of a plan (delta 0, the diagonal, is
// in group 0).
inline void sym_group(const SymPlan &pl, int g, int *d_lo, int *d_hi)
{
    *d_lo = g == 0 ? 0 : 1 + g * pl.G;
    const int hi = 1 + (g + 1) * pl.G;
    *d_hi = hi < pl.M / 2 + 1 ? hi : pl.M / 2 + 1;
}

// Library workspace allowed for one pair-once evaluation of n particles
// (partials and running sum) before the ring is split into more groups:
// 1 GiB, or 16 float4 slots per particle where that is more (n > 2^22).
// The environment variable NBODY_SYM_WORKSPACE=<bytes> sets another limit
// (tests use it to split small rings into many groups).
inline size_t sym_workspace_budget(int64_t n)
{
    if (const char *env = std::getenv("NBODY_SYM_WORKSPACE")) {
        const unsigned long long v = std::strtoull(env, nullptr, 10);
        if (v > 0) return (size_t)v;
    }
    const size_t slots16 = 256 * (size_t)n;
    return slots16 > ((size_t)1 << 30) ? slots16 : ((size_t)1 << 30);
}

// Number of tiles of block I in ring group [d_lo, d_hi): the TPB diagonal
// tiles when d_lo == 0, then TPB tiles per ring delta the block meets.
__host__ __device__ __forceinline__ int group_tiles(int I, int M, int d_lo, int d_hi, int TPB)
{
    const int dj = group_first_delta(d_lo);
    const int hi = min(d_hi - 1, ring_len(I, M));
    return (d_lo == 0 ? TPB : 0) + (hi >= dj ? (hi - dj + 1) * TPB : 0);
}

// Tile u of block I's sequence in ring group [d_lo, ...): the TPB diagonal
// tiles (delta 0) when the group holds them, then the ring tiles
// delta-major.  Returns the first particle index of the tile.
template <int PB>
__device__ __forceinline__ int tile_base(int u, int I, int M, int d_lo, int &delta)
{
    constexpr int TPB = PB / 64;
    if (d_lo == 0) {
        if (u < TPB) {
            delta = 0;
            return I * PB + u * 64;
        }
        u -= TPB;
    }
    const int q = u / TPB;
    delta = group_first_delta(d_lo) + q;
    int J = I + delta;
    if (J >= M) J -= M;
    return J * PB + (u - q * TPB) * 64;
}

__device__ __forceinline__ float4 load_particle(const float *__restrict__ x,
                                                const float *__restrict__ m, int j, int n)
{
    return (j < n) ? make_float4(x[3 * j], x[3 * j + 1], x[3 * j + 2], m[j])
                   : make_float4(kPadCol, kPadCol, kPadCol, 0.0f);
}

// One pair met once: i-side added to (tx, ty, tz, tp); j-side added to
// (gx, gy, gz, gp), or stored there when FIRST (the first row of a step).
template <bool FIRST>
__device__ __forceinline__ void pair_once_term(float xi, float yi, float zi, float mi, float4 q,
                                               float eps2, float &tx, float &ty, float &tz,
                                               float &tp, float &gx, float &gy, float &gz,
                                               float &gp)
{
    const float dx = xi - q.x;
    const float dy = yi - q.y;
    const float dz = zi - q.z;
    float s2 = __builtin_fmaf(dx, dx, eps2);
    s2 = __builtin_fmaf(dy, dy, s2);
    s2 = __builtin_fmaf(dz, dz, s2);
    const float r = __builtin_amdgcn_rsqf(s2);
    const float r3 = r * (r * r);
    // i-side: + m_j r^3 d, + m_j r
    const float f = q.w * r3;
    tp = __builtin_fmaf(q.w, r, tp);
    tx = __builtin_fmaf(f, dx, tx);
    ty = __builtin_fmaf(f, dy, ty);
    tz = __builtin_fmaf(f, dz, tz);
    // j-side: - m_i r^3 d, + m_i r
    const float g = mi * r3;
    if (FIRST) {
        gx = -g * dx;
        gy = -g * dy;
        gz = -g * dz;
        gp = mi * r;
    } else {
        gx = __builtin_fmaf(-g, dx, gx);
        gy = __builtin_fmaf(-g, dy, gy);
        gz = __builtin_fmaf(-g, dz, gz);
        gp = __builtin_fmaf(mi, r, gp);
    }
}

// One pair of a ring tile: i-side added to (tx, ty, tz, tp), j-side added
// to the slot value g (the chain of a step's K rows starts from the slot,
// so no separate add folds it in).  POT false: the caller stores no
// potential, and its two terms (2 of the pair's 19 instructions) are not
// formed.
template <bool POT = true>
__device__ __forceinline__ void pair_once_fold(float xi, float yi, float zi, float mi, float4 q,
                                               float eps2, float &tx, float &ty, float &tz,
                                               float &tp, float4 &g)
{
    const float dx = xi - q.x;
    const float dy = yi - q.y;
    const float dz = zi - q.z;
    float s2 = __builtin_fmaf(dx, dx, eps2);
    s2 = __builtin_fmaf(dy, dy, s2);
    s2 = __builtin_fmaf(dz, dz, s2);
    const float r = __builtin_amdgcn_rsqf(s2);
    const float r3 = r * (r * r);
    const float f = q.w * r3;
    if (POT) tp = __builtin_fmaf(q.w, r, tp);
    tx = __builtin_fmaf(f, dx, tx);
    ty = __builtin_fmaf(f, dy, ty);
    tz = __builtin_fmaf(f, dz, tz);
    const float h = mi * r3;
    g.x = __builtin_fmaf(-h, dx, g.x);
    g.y = __builtin_fmaf(-h, dy, g.y);
    g.z = __builtin_fmaf(-h, dz, g.z);
    if (POT) g.w = __builtin_fmaf(mi, r, g.w);
}

// The 64 steps of a ring tile for one wave: lane l meets the particle in
// tile entry l + s at step s and adds its j-side terms to slot l + s.
// `tile` has kTileLds entries (the tile twice), `slot` this wave's
// kSlotLds slots.
// PARTIAL: only the first kv row groups of the wave hold particles (the
// last block of a system); the others are padding with mass 0, whose terms
// are exactly zero on both sides, so skipping them changes no bit.
template <int K, bool PARTIAL = false, bool POT = true>
__device__ __forceinline__ void ring_tile_steps(const float (&xi)[K], const float (&yi)[K],
                                                const float (&zi)[K], const float (&mi)[K],
                                                const float4 *tile, float4 *slot, int lane,
                                                float eps2, float (&tx)[K], float (&ty)[K],
                                                float (&tz)[K], float (&tp)[K], int kv = K)
{
    const float4 *tq = tile + lane;
    float4 *sl = slot + lane;
    float4 q = tq[0];
#pragma unroll 8
    for (int s = 0; s < 64; ++s) {
        // Compiler-only barrier: this step's slot read stays after the
        // previous step's slot write (another lane wrote the slot read here).
        __asm__ volatile("" ::: "memory");
        float4 g = sl[s];
        const float4 qn = tq[s + 1];  // next step's particle (read-only tile)
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (!PARTIAL || k < kv)
                pair_once_fold<POT>(xi[k], yi[k], zi[k], mi[k], q, eps2, tx[k], ty[k], tz[k], tp[k],
                               g);
        sl[s] = g;
        q = qn;
    }
    // particle e collected in slots e and e + 64: fold them into slot e
    __asm__ volatile("" ::: "memory");
    const float4 lo = slot[lane];
    const float4 hi = slot[lane + 64];
    slot[lane] = make_float4(lo.x + hi.x, lo.y + hi.y, lo.z + hi.z, lo.w + hi.w);
}

// One step s of a diagonal tile: rows k < R meet entry l + s pair-once.
template <int K, int R, bool POT = true>
__device__ __forceinline__ void diag_step(const float (&xi)[K], const float (&yi)[K],
                                          const float (&zi)[K], const float (&mi)[K],
                                          const float4 *tq, float4 *sl, int s, float eps2,
                                          float (&tx)[K], float (&ty)[K], float (&tz)[K],
                                          float (&tp)[K])
{
    if constexpr (R > 0) {
        // keep this step's slot read after the previous step's slot write
        __asm__ volatile("" ::: "memory");
        const float4 q = tq[s];
        float4 g = sl[s];
#pragma unroll
        for (int k = 0; k < R; ++k)
            pair_once_fold<POT>(xi[k], yi[k], zi[k], mi[k], q, eps2, tx[k], ty[k], tz[k], tp[k], g);
        sl[s] = g;
    }
}

// Diagonal tile whose rows are this wave's row group KT (rows k < KT belong
// to earlier tiles of the block and meet it pair-once; rows k > KT to later
// ones, which meet it from their side).  Row group KT meets its own tile
// pair-once too: lane l and particle l + s (mod 64) form each unordered
// pair once for s = 1..31, and for s = 32 the pair {l, l + 32} is met by
// both lanes, so each takes its i-side only; s = 0 (the particle itself)
// and s = 33..63 (met as 64 - s by the partner) are skipped.  The j-side
// sums fill this wave's slots like a ring tile's and are folded to slot e.
template <int K, int KT, bool POT = true>
__device__ __forceinline__ void diag_self_steps(const float (&xi)[K], const float (&yi)[K],
                                                const float (&zi)[K], const float (&mi)[K],
                                                const float4 *tile, float4 *slot, int lane,
                                                float eps2, float (&tx)[K], float (&ty)[K],
                                                float (&tz)[K], float (&tp)[K])
{
    const float4 *tq = tile + lane;
    float4 *sl = slot + lane;
    // The loops run two steps per trip and are kept rolled: fully unrolled,
    // the K instances of this function made a kernel larger than the
    // instruction cache and slowed its ring loop.
    diag_step<K, KT, POT>(xi, yi, zi, mi, tq, sl, 0, eps2, tx, ty, tz, tp);
#pragma nounroll
    for (int s = 1; s < 31; s += 2) {
        diag_step<K, KT + 1, POT>(xi, yi, zi, mi, tq, sl, s, eps2, tx, ty, tz, tp);
        diag_step<K, KT + 1, POT>(xi, yi, zi, mi, tq, sl, s + 1, eps2, tx, ty, tz, tp);
    }
    diag_step<K, KT + 1, POT>(xi, yi, zi, mi, tq, sl, 31, eps2, tx, ty, tz, tp);
    diag_step<K, KT, POT>(xi, yi, zi, mi, tq, sl, 32, eps2, tx, ty, tz, tp);
    pair_term(xi[KT], yi[KT], zi[KT], tq[32], eps2, tx[KT], ty[KT], tz[KT], tp[KT]);
    if (KT > 0) {
#pragma nounroll
        for (int s = 33; s < 63; s += 2) {
            diag_step<K, KT, POT>(xi, yi, zi, mi, tq, sl, s, eps2, tx, ty, tz, tp);
            diag_step<K, KT, POT>(xi, yi, zi, mi, tq, sl, s + 1, eps2, tx, ty, tz, tp);
        }
        diag_step<K, KT, POT>(xi, yi, zi, mi, tq, sl, 63, eps2, tx, ty, tz, tp);
    }
    __asm__ volatile("" ::: "memory");
    const float4 lo = slot[lane];
    const float4 hi = slot[lane + 64];
    slot[lane] = make_float4(lo.x + hi.x, lo.y + hi.y, lo.z + hi.z, lo.w + hi.w);
}

template <int K, int KT = 0, bool POT = true>
__device__ __forceinline__ void diag_tile_dispatch(int kt, const float (&xi)[K],
                                                   const float (&yi)[K], const float (&zi)[K],
                                                   const float (&mi)[K], const float4 *tile,
                                                   float4 *slot, int lane, float eps2,
                                                   float (&tx)[K], float (&ty)[K], float (&tz)[K],
                                                   float (&tp)[K])
{
    if (kt == KT)
        diag_self_steps<K, KT, POT>(xi, yi, zi, mi, tile, slot, lane, eps2, tx, ty, tz, tp);
    else if constexpr (KT + 1 < K)
        diag_tile_dispatch<K, KT + 1, POT>(kt, xi, yi, zi, mi, tile, slot, lane, eps2, tx, ty, tz, tp);
}

// The 64 steps of one tile for one wave.  Lane l meets tile particle
// (l + s) mod 64 at step s.  Ring tiles (DIAG false): every row tile meets
// the tile pair-once.  Diagonal tile t (DIAG true): row tile a = a0 + k
// meets it pair-once if a < t, as masked ordered pairs if a == t, not at all
// if a > t.  j-side sums go to this wave's LDS slots (read-modify-write).
template <int K, bool DIAG>
__device__ __forceinline__ void tile_steps(const float (&xi)[K], const float (&yi)[K],
                                           const float (&zi)[K], const float (&mi)[K],
                                           const int (&ii)[K], const float4 *tile, float4 *slot,
                                           int lane, int a0, int t, int jbase, float eps2,
                                           float (&tx)[K], float (&ty)[K], float (&tz)[K],
                                           float (&tp)[K])
{
    const bool any_once = !DIAG || a0 < t;
    float4 q = tile[lane];
    for (int s = 0; s < 64; ++s) {
        const int jj = (lane + s) & 63;
        // Compiler-only barrier: this step's slot read stays after the
        // previous step's slot write (another lane may have written it).
        __asm__ volatile("" ::: "memory");
        float4 ja = make_float4(0.f, 0.f, 0.f, 0.f);
        if (any_once) ja = slot[jj];
        const float4 qn = tile[(jj + 1) & 63];  // next step's particle (read-only tile)
        float gx = 0.f, gy = 0.f, gz = 0.f, gp = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!DIAG) {
                if (k == 0)
                    pair_once_term<true>(xi[k], yi[k], zi[k], mi[k], q, eps2, tx[k], ty[k], tz[k],
                                         tp[k], gx, gy, gz, gp);
                else
                    pair_once_term<false>(xi[k], yi[k], zi[k], mi[k], q, eps2, tx[k], ty[k], tz[k],
                                          tp[k], gx, gy, gz, gp);
            } else if (a0 + k < t) {
                pair_once_term<false>(xi[k], yi[k], zi[k], mi[k], q, eps2, tx[k], ty[k], tz[k],
                                      tp[k], gx, gy, gz, gp);
            } else if (a0 + k == t) {
                pair_term_masked(xi[k], yi[k], zi[k], q, eps2, jbase + jj == ii[k], tx[k], ty[k],
                                 tz[k], tp[k]);
            }
        }
        if (any_once) {
            ja.x += gx;
            ja.y += gy;
            ja.z += gz;
            ja.w += gp;
            slot[jj] = ja;
        }
        q = qn;
    }
}

// One workgroup of W*64 lanes evaluates chunk c of block I.  x, m and
// partial are the system's own arrays (offsets already applied).  tile and
// jacc are the workgroup's LDS buffers.  Starts with a workgroup barrier, so
// the LDS buffers may be reused by consecutive calls.
//
// Diagonal tiles are pair-once too (for W <= 8; larger blocks meet them as
// masked ordered pairs): the rows of lane-slot k of wave wv form
// the block's tile a = wv*K + k.  On diagonal tile t, row tile a < t meets
// it pair-once, a == t meets it as ordered pairs with j == i removed by
// index (one-wave blocks: pair-once within the tile, diag_self_steps), and
// a > t skips it (that pair of tiles is met on diagonal tile a).
// The j-side sums of a diagonal tile belong to rows of the same block; the
// wave that holds tile t's rows adds them to its own accumulators.
// POT false: no potential is stored, and the ring and one-wave diagonal
// tiles do not form its terms (the partials' w component is then partial).
// SKIP_PAD: skip the ring-tile work of row groups that hold only padding
// (bitwise neutral: their terms are exactly zero).  Worth it for ensembles
// of small systems, where a last block is often part padding (5% of the
// row-group work on the 4,096-system ensemble); single systems keep the
// lighter loop.
template <int W, int K, bool SKIP_PAD = false, bool POT = true>
__device__ __forceinline__ void pair_once_block(const float *__restrict__ x,
                                                const float *__restrict__ m, int n, float eps2,
                                                int M, int I, int c, int C, int d_lo, int d_hi,
                                                float4 *partial, float4 *tile,
                                                float4 (*jacc)[kSlotLds])
{
    constexpr int PB = W * 64 * K;   // particles per block
    constexpr int TPB = PB / 64;     // 64-particle tiles per block
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;

    // ---- own rows
    float xi[K], yi[K], zi[K], mi[K];
    int ii[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = I * PB + wv * 64 * K + k * 64 + lane;
        ii[k] = i;
        if (i < n) {
            xi[k] = x[3 * i];
            yi[k] = x[3 * i + 1];
            zi[k] = x[3 * i + 2];
            mi[k] = m[i];
        } else {
            xi[k] = yi[k] = zi[k] = kPadRow;
            mi[k] = 0.0f;
        }
    }
    float ax[K], ay[K], az[K], ap[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ax[k] = ay[k] = az[k] = ap[k] = 0.0f;
    // row groups of this wave that hold particles (K except in a last block)
    const int kv = SKIP_PAD ? min(K, max(0, (n - (I * PB + wv * 64 * K) + 63) / 64)) : K;

    // ---- this chunk's share of the block's tile sequence in the group;
    // tiles that hold only padding are skipped (uniform).
    const int U = group_tiles(I, M, d_lo, d_hi, TPB);
    const int dj = group_first_delta(d_lo);
    const int u0 = (int)((long long)U * c / C);
    const int u1 = (int)((long long)U * (c + 1) / C);
    // Small workgroups prefetch the next tile into registers while the
    // current one is consumed; 16-wave blocks (one per CU, 128 VGPRs) have
    // no registers to spare and rely on the other waves to hide the load.
    constexpr bool kPrefetch = (W <= 8);
    // Diagonal tiles pair-once (halves their work) where registers allow;
    // 16-wave blocks meet them as masked ordered pairs (at 2^17 particles
    // and up the diagonal is under 1/32 of the pairs).
    constexpr bool kOnceDiag = (W <= 8);
    // One-wave blocks (ensembles of small systems, mid-size single systems,
    // where diagonal tiles are a fifth of the work) also meet each diagonal
    // tile's own 64 particles pair-once (diag_self_steps).  Wider blocks
    // keep the masked ordered self tile: there the diagonal is rare, and
    // the larger code changed the schedule of their ring loop (6-8% slower
    // at 2^20 bodies).
    constexpr bool kSelfDiag = (W == 1);
    int u = u0, delta = 0, jbase = 0;
    for (; u < u1; ++u)
        if ((jbase = tile_base<PB>(u, I, M, d_lo, delta)) < n) break;
    float4 next = make_float4(0.f, 0.f, 0.f, 0.f);
    if (kPrefetch && u < u1 && tid < 64) next = load_particle(x, m, jbase + tid, n);

    while (u < u1) {
        // previous tile and its j-slot sums are done (and the LDS buffers
        // free on entry: callers may loop over blocks)
        __syncthreads();
        if (tid < 64) {
            const float4 v = kPrefetch ? next : load_particle(x, m, jbase + tid, n);
            tile[tid] = v;
            tile[tid + 64] = v;
        }
        jacc[wv][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        jacc[wv][lane + 64] = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        const int cur_u = u, cur_delta = delta, cur_base = jbase;
        for (++u; u < u1; ++u)
            if ((jbase = tile_base<PB>(u, I, M, d_lo, delta)) < n) break;
        if (kPrefetch && u < u1 && tid < 64) next = load_particle(x, m, jbase + tid, n);

        float tx[K], ty[K], tz[K], tp[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tx[k] = ty[k] = tz[k] = tp[k] = 0.0f;

        const int t = cur_u;                         // diagonal tile index when cur_delta == 0
        const bool diag = (cur_delta == 0);
        float4 *slot = &jacc[wv][0];
        if (!diag) {
            if (!SKIP_PAD || kv == K)
                ring_tile_steps<K, false, POT>(xi, yi, zi, mi, tile, slot, lane, eps2, tx, ty, tz, tp);
            else if (kv > 0)
                ring_tile_steps<K, true, POT>(xi, yi, zi, mi, tile, slot, lane, eps2, tx, ty, tz, tp,
                                         kv);
        } else if constexpr (kSelfDiag) {
            // one wave: its row group k is the block's tile k, so diagonal
            // tile t meets row groups k < t pair-once and row group t itself
            diag_tile_dispatch<K, 0, POT>(t, xi, yi, zi, mi, tile, slot, lane, eps2, tx, ty, tz, tp);
        } else if (kOnceDiag) {
            tile_steps<K, true>(xi, yi, zi, mi, ii, tile, slot, lane, wv * K, t, cur_base, eps2, tx,
                                ty, tz, tp);
        } else {
            // ordered pairs, i-side only, j == i removed by index
            for (int s = 0; s < 64; ++s) {
                const float4 q = tile[s];
                const int j = cur_base + s;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    pair_term_masked(xi[k], yi[k], zi[k], q, eps2, j == ii[k], tx[k], ty[k], tz[k],
                                     tp[k]);
            }
        }
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < K; ++k) {
            ax[k] += tx[k];
            ay[k] += ty[k];
            az[k] += tz[k];
            ap[k] += tp[k];
        }
        __syncthreads();  // every wave's j-side slots are complete
        if (!diag) {
            if (tid < 64) {
                // particle tid: every wave folded its slot tid + 64 into slot
                // tid (ring_tile_steps); add the waves' slots in wave order
                float4 sum = jacc[0][tid];
#pragma unroll
                for (int w2 = 1; w2 < W; ++w2) {
                    const float4 v = jacc[w2][tid];
                    sum.x += v.x;
                    sum.y += v.y;
                    sum.z += v.z;
                    sum.w += v.w;
                }
                const int j = cur_base + tid;
                if (j < n) partial[(size_t)(C + cur_delta - dj) * n + j] = sum;
            }
        } else if (kOnceDiag && wv == t / K) {
            // this wave holds diagonal tile t's rows (lane-slot t % K); the
            // diagonal steps leave their sums in slots 0..63
            float4 sum = jacc[0][lane];
#pragma unroll
            for (int w2 = 1; w2 < W; ++w2) {
                const float4 v = jacc[w2][lane];
                sum.x += v.x;
                sum.y += v.y;
                sum.z += v.z;
                sum.w += v.w;
            }
            const int kt = t - wv * K;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k == kt) {
                    ax[k] += sum.x;
                    ay[k] += sum.y;
                    az[k] += sum.z;
                    ap[k] += sum.w;
                }
        }
    }

#pragma unroll
    for (int k = 0; k < K; ++k)
        if (ii[k] < n) partial[(size_t)c * n + ii[k]] = make_float4(ax[k], ay[k], az[k], ap[k]);
}

}  // namespace nbody
