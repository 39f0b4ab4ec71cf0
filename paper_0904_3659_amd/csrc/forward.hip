// Forward evaluation of Eq. (gravity) (Sec. I): a_i and p_i for every i,
// j != i, float32, on gfx950.
//
// Work decomposition
//   grid.x  : i-blocks of BLOCK*K particles; lane t of the workgroup keeps
//             particles i0 + k*BLOCK + t (k < K) and their accumulators in
//             VGPRs (the register-resident i-block; the paper's i-loop
//             unrolling of Fig. sim-u, Sec. IV-A).
//   grid.y  : j-splits; split s sums j in [s*chunk, min(n, (s+1)*chunk)).
//             With more than one split, each writes a float4 partial
//             (ax, ay, az, p) per i and a second kernel adds the splits in
//             fixed order.
//   j-tiles : BLOCK consecutive j are staged into LDS as float4 (x, y, z, m)
//             -- the packing of x[n][3], m[n] happens here, one coalesced
//             load per lane -- and read back by every lane as a broadcast.
//             The next tile is fetched into registers while the current
//             one is consumed.  The inner loop is unrolled U times over j
//             (the paper's j-unrolling of Fig. double-u).
//   accuracy: each tile's contribution is summed in fresh registers and
//             folded into the running sum once per tile (two-level
//             accumulation), which keeps the float32 error flat in n.
//   self    : only tiles that intersect the workgroup's own i-range, and
//             the ragged last tile, take the masked loop (index compare);
//             every other tile runs unmasked.
//
// No atomics: the result is bitwise reproducible for a given variant, n
// and split count.
#include "common.hpp"
#include "pair_once.hpp"
#include "wave_sum.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <type_traits>

namespace nbody {
namespace {

struct FwdArgs {
    const float *x;
    const float *m;
    int n;
    float eps2;
    int chunk;        // j per split (a multiple of the tile size)
    float4 *partial;  // [splits][n] when PARTIAL
    float *a;
    float *p;
    double *partial_d;  // [splits][n][4] when PARTIAL and D64
};

// D64: the running sums of every row are float64; each j-tile's float32
// partial is widened and added once per tile, and split partials are kept
// and added in float64.  Only the float32 sums inside one tile remain, so
// the rounding error no longer grows with the number of tiles (n / BLOCK).
// About 8 float64 VALU operations per row per tile: under 1% of the pair
// work at BLOCK = 64.
template <int BLOCK, int K, int U, bool PARTIAL, bool D64 = false>
__global__ __launch_bounds__(BLOCK) void forward_kernel(FwdArgs P)
{
    using Acc = typename std::conditional<D64, double, float>::type;
    constexpr int TILE = BLOCK;
    __shared__ float4 tile[TILE];

    const int tid = threadIdx.x;
    const int n = P.n;
    const int i0 = blockIdx.x * (BLOCK * K);
    const int jbeg = blockIdx.y * P.chunk;
    const int jend = min(n, jbeg + P.chunk);
    const float eps2 = P.eps2;

    float xi[K], yi[K], zi[K];
    int ii[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = i0 + k * BLOCK + tid;
        ii[k] = i;
        const int ic = i < n ? i : n - 1;  // idle lanes mirror a valid row
        xi[k] = P.x[3 * ic + 0];
        yi[k] = P.x[3 * ic + 1];
        zi[k] = P.x[3 * ic + 2];
    }
    Acc ax[K], ay[K], az[K], pp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ax[k] = ay[k] = az[k] = pp[k] = Acc(0);

    // j-tile prefetch registers
    float4 next = make_float4(0.f, 0.f, 0.f, 0.f);
    {
        const int j = jbeg + tid;
        if (j < jend) next = make_float4(P.x[3 * j], P.x[3 * j + 1], P.x[3 * j + 2], P.m[j]);
    }

    const int iblk_end = i0 + BLOCK * K;
    for (int t0 = jbeg; t0 < jend; t0 += TILE) {
        __syncthreads();  // previous tile fully consumed
        tile[tid] = next;
        __syncthreads();
        {
            const int j = t0 + TILE + tid;
            next = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < jend) next = make_float4(P.x[3 * j], P.x[3 * j + 1], P.x[3 * j + 2], P.m[j]);
        }

        float tx[K], ty[K], tz[K], tp[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tx[k] = ty[k] = tz[k] = tp[k] = 0.0f;

        const int cnt = min(TILE, jend - t0);
        const bool masked = (cnt < TILE) || (t0 < iblk_end && t0 + TILE > i0);
        if (!masked) {
            for (int jj = 0; jj < TILE; jj += U) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const float4 q = tile[jj + u];
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        pair_term(xi[k], yi[k], zi[k], q, eps2, tx[k], ty[k], tz[k], tp[k]);
                }
            }
        } else {
            for (int jj = 0; jj < cnt; ++jj) {
                const float4 q = tile[jj];
                const int j = t0 + jj;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    pair_term_masked(xi[k], yi[k], zi[k], q, eps2, j == ii[k], tx[k], ty[k],
                                     tz[k], tp[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            ax[k] += Acc(tx[k]);
            ay[k] += Acc(ty[k]);
            az[k] += Acc(tz[k]);
            pp[k] += Acc(tp[k]);
        }
    }

#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = ii[k];
        if (i >= n) continue;
        if (PARTIAL && D64) {
            double2 *q = reinterpret_cast<double2 *>(P.partial_d + ((size_t)blockIdx.y * n + i) * 4);
            q[0] = make_double2(ax[k], ay[k]);
            q[1] = make_double2(az[k], pp[k]);
        } else if (PARTIAL) {
            P.partial[(size_t)blockIdx.y * n + i] =
                make_float4((float)ax[k], (float)ay[k], (float)az[k], (float)pp[k]);
        } else {
            P.a[3 * i + 0] = (float)ax[k];
            P.a[3 * i + 1] = (float)ay[k];
            P.a[3 * i + 2] = (float)az[k];
            if (P.p) P.p[i] = (float)pp[k];
        }
    }
}

// Sum the split partials of each row in split order and store a, p.
__global__ __launch_bounds__(256) void reduce_splits_kernel(const float4 *__restrict__ partial,
                                                            int splits, int n, float *a, float *p)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float4 s = partial[i];
    for (int k = 1; k < splits; ++k) {
        const float4 q = partial[(size_t)k * n + i];
        s.x += q.x;
        s.y += q.y;
        s.z += q.z;
        s.w += q.w;
    }
    a[3 * i + 0] = s.x;
    a[3 * i + 1] = s.y;
    a[3 * i + 2] = s.z;
    if (p) p[i] = s.w;
}

// The float64 form of reduce_splits_kernel (partials of D64 kernels).
__global__ __launch_bounds__(256) void reduce_splits_d_kernel(const double *__restrict__ partial,
                                                              int splits, int n, float *a, float *p)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double2 *q = reinterpret_cast<const double2 *>(partial);
    double2 s0 = q[2 * (size_t)i], s1 = q[2 * (size_t)i + 1];
    for (int k = 1; k < splits; ++k) {
        const size_t e = 2 * ((size_t)k * n + i);
        const double2 t0 = q[e], t1 = q[e + 1];
        s0.x += t0.x;
        s0.y += t0.y;
        s1.x += t1.x;
        s1.y += t1.y;
    }
    a[3 * i + 0] = (float)s0.x;
    a[3 * i + 1] = (float)s0.y;
    a[3 * i + 2] = (float)s1.x;
    if (p) p[i] = (float)s1.y;
}

// ---------------------------------------------------------------------------
// One-launch split gather for small n, where launch latency and not the
// pairs sets the time.  A workgroup of W waves owns 64 rows (one per lane,
// the same rows in every wave) and splits j among its waves; S such
// workgroups per row block along grid.y spread the j-range over the chip.
// Workgroup (b, s) owns rows [64 b, 64 b + 64) and its wave w sums
// j in [(s W + w) chunk, (s W + w + 1) chunk) through a wave-private LDS
// tile.  The W wave sums are added in wave order through LDS; with S = 1
// they are the result, otherwise they are stored as the split's float4
// partial and the last workgroup of row block b to arrive (a ticket counter
// per row block) adds the S partials in split order, stores a, p and puts
// the counter back to zero for the next launch.  Which workgroup arrives
// last varies from run to run, but the order of every addition does not:
// the result is bitwise reproducible for a given n, W and S.
//
// The agent-scope fences around the ticket write back and invalidate the
// XCD's L2, so the scheme pays off only with few workgroups: the same tail
// on the 256-row split gather (about 1000 workgroups at n = 7500) ran 3x
// slower than its reduction launch.
struct LaArgs {
    const float *x;
    const float *m;
    int n;
    float eps2;
    int chunk;        // j per wave
    int splits;       // S (grid.y)
    float4 *partial;  // [S][n] when S > 1
    int *ctr;         // [grid.x] tickets, zero between launches
    float *a;
    float *p;
};

template <int W>
__global__ __launch_bounds__(W * 64) void forward_la_kernel(LaArgs P)
{
    __shared__ float4 tiles[W][64];
    __shared__ float4 red[W][64];
    __shared__ int last;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int n = P.n;
    const float eps2 = P.eps2;
    const int row0 = blockIdx.x * 64;
    const int i = row0 + lane;
    const int ic = i < n ? i : n - 1;
    const float xi = P.x[3 * ic], yi = P.x[3 * ic + 1], zi = P.x[3 * ic + 2];
    const int64_t jb64 = ((int64_t)blockIdx.y * W + wv) * P.chunk;
    const int jb = (int)min<int64_t>(jb64, n);
    const int je = min(n, jb + P.chunk);
    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
    float4 *tile = tiles[wv];
    for (int t0 = jb; t0 < je; t0 += 64) {
        const int j = t0 + lane;
        // wave-private tile: compiler-only barriers keep the previous tile's
        // reads before this write and this write before the reads below
        __asm__ volatile("" ::: "memory");
        tile[lane] = (j < je) ? make_float4(P.x[3 * j], P.x[3 * j + 1], P.x[3 * j + 2], P.m[j])
                              : make_float4(0.f, 0.f, 0.f, 0.f);
        __asm__ volatile("" ::: "memory");
        float tx = 0.f, ty = 0.f, tz = 0.f, tp = 0.f;
        const int cnt = min(64, je - t0);
        if (cnt == 64 && (t0 >= row0 + 64 || t0 + 64 <= row0)) {
#pragma unroll 8
            for (int q = 0; q < 64; ++q) pair_term(xi, yi, zi, tile[q], eps2, tx, ty, tz, tp);
        } else {
            for (int q = 0; q < cnt; ++q)
                pair_term_masked(xi, yi, zi, tile[q], eps2, t0 + q == i, tx, ty, tz, tp);
        }
        ax += tx;
        ay += ty;
        az += tz;
        ap += tp;
    }
    red[wv][lane] = make_float4(ax, ay, az, ap);
    __syncthreads();
    if (P.splits == 1) {
        if (wv == 0 && i < n) {
            float4 t = red[0][lane];
#pragma unroll
            for (int w2 = 1; w2 < W; ++w2) {
                const float4 q = red[w2][lane];
                t.x += q.x;
                t.y += q.y;
                t.z += q.z;
                t.w += q.w;
            }
            P.a[3 * i + 0] = t.x;
            P.a[3 * i + 1] = t.y;
            P.a[3 * i + 2] = t.z;
            if (P.p) P.p[i] = t.w;
        }
        return;
    }
    if (wv == 0) {
        float4 t = red[0][lane];
#pragma unroll
        for (int w2 = 1; w2 < W; ++w2) {
            const float4 q = red[w2][lane];
            t.x += q.x;
            t.y += q.y;
            t.z += q.z;
            t.w += q.w;
        }
        if (i < n) P.partial[(size_t)blockIdx.y * n + i] = t;
        __threadfence();  // release the partial before taking a ticket
    }
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(&P.ctr[blockIdx.x], 1) == P.splits - 1);
    __syncthreads();
    if (!last || wv != 0) return;
    __threadfence();  // acquire every other split's partial
    if (i < n) {
        float4 t = P.partial[i];
        for (int k = 1; k < P.splits; ++k) {
            const float4 q = P.partial[(size_t)k * n + i];
            t.x += q.x;
            t.y += q.y;
            t.z += q.z;
            t.w += q.w;
        }
        P.a[3 * i + 0] = t.x;
        P.a[3 * i + 1] = t.y;
        P.a[3 * i + 2] = t.z;
        if (P.p) P.p[i] = t.w;
    }
    if (lane == 0) atomicExch(&P.ctr[blockIdx.x], 0);
}

// ---------------------------------------------------------------------------
// Row-per-wave kernel for the smallest n (up to a few thousand bodies),
// where one call costs launch latency plus its longest chain of dependent
// steps rather than pairs.  Wave w owns rows [K w, K w + K): their
// positions are the same for every lane (scalar registers) and lane l sums
// j = l, l + 64, l + 128, ... for all K rows.  The 64 lane sums of a row
// are then added by a fixed butterfly (DPP within rows of 16 lanes, then
// two lane swaps), so every lane ends with the same, bitwise reproducible
// total.  No LDS tile, no partials, no ticket and no second launch: at
// n = 1,024 with K = 1 the 1,024 waves give every SIMD of the chip one.
struct RowArgs {
    const float *x;
    const float *m;
    int n;
    float eps2;
    float *a;
    float *p;
};

template <int K>
__global__ __launch_bounds__(256) void forward_row_kernel(RowArgs P)
{
    const int n = P.n;
    const float eps2 = P.eps2;
    const int lane = threadIdx.x & 63;
    const int i0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6))) * K;
    if (i0 >= n) return;  // the whole wave: no barrier follows
    float xi[K], yi[K], zi[K], ax[K], ay[K], az[K], ap[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int ik = min(i0 + k, n - 1);  // rows past n are computed, not stored
        xi[k] = P.x[3 * ik];
        yi[k] = P.x[3 * ik + 1];
        zi[k] = P.x[3 * ik + 2];
        ax[k] = ay[k] = az[k] = ap[k] = 0.f;
    }
#pragma unroll 4
    for (int j = lane; j < n; j += 64) {
        const float4 q = make_float4(P.x[3 * j], P.x[3 * j + 1], P.x[3 * j + 2], P.m[j]);
#pragma unroll
        for (int k = 0; k < K; ++k)
            pair_term_masked(xi[k], yi[k], zi[k], q, eps2, j == i0 + k, ax[k], ay[k], az[k], ap[k]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        ax[k] = wave_sum(ax[k]);
        ay[k] = wave_sum(ay[k]);
        az[k] = wave_sum(az[k]);
        ap[k] = wave_sum(ap[k]);
    }
    // lane k stores row i0 + k
    float sx = ax[0], sy = ay[0], sz = az[0], sp = ap[0];
#pragma unroll
    for (int k = 1; k < K; ++k)
        if (lane == k) {
            sx = ax[k];
            sy = ay[k];
            sz = az[k];
            sp = ap[k];
        }
    const int i = i0 + lane;
    if (lane < K && i < n) {
        P.a[3 * i + 0] = sx;
        P.a[3 * i + 1] = sy;
        P.a[3 * i + 2] = sz;
        if (P.p) P.p[i] = sp;
    }
}

using RowFn = void (*)(RowArgs);

using LaFn = void (*)(LaArgs);

using KernelFn = void (*)(FwdArgs);

// A variant is either a gather kernel (every ordered pair, rows own all j)
// or, when sym_w > 0, the pair-once kernel of forward_sym.hip with W waves
// and K rows per lane.
struct Variant {
    const char *name;
    int block, k, unroll;
    KernelFn direct, partial;
    int sym_w, sym_k, sym_occ, sym_rounds;
    LaFn la;  // one-launch split gather (wave-split workgroups x S splits)
    int la_w;
    bool d64;     // float64 running sums (forward_kernel's D64)
    bool la_one;  // one-launch kernel with a single split: no partials, no ticket
    RowFn row;    // row-per-wave kernel (K = row_k rows per wave)
    int row_k;
};

#define FWD_VARIANT(B, K, U) \
    {"fwd_b" #B "_k" #K "_u" #U, B, K, U, forward_kernel<B, K, U, false>, forward_kernel<B, K, U, true>, 0, 0, 0, 1, nullptr, 0, false, false}
#define FWD_D64_VARIANT(B, K, U)                                                               \
    {"fwd_b" #B "_k" #K "_u" #U "_f64sum", B, K, U, forward_kernel<B, K, U, false, true>,      \
     forward_kernel<B, K, U, true, true>, 0, 0, 0, 1, nullptr, 0, true, false}
#define FWD_SYM_VARIANT(W, K, O) {"fwd_sym_w" #W "_k" #K "_o" #O, 0, 0, 0, nullptr, nullptr, W, K, O, 1, nullptr, 0, false, false}
// Pair-once blocks in R rounds of workgroups (R times the chunks).
#define FWD_SYM_R_VARIANT(W, K, R) {"fwd_sym_w" #W "_k" #K "_r" #R, 0, 0, 0, nullptr, nullptr, W, K, 1, R, nullptr, 0, false, false}
#define FWD_LA_VARIANT(W) {"fwd_la_w" #W, 64, 1, 0, nullptr, nullptr, 0, 0, 0, 1, forward_la_kernel<W>, W, false, false}
// The same kernel with one split: the W waves of a row block's workgroup
// share all of j, and their wave-ordered sum is the result.
#define FWD_LA1_VARIANT(W) {"fwd_la1_w" #W, 64, 1, 0, nullptr, nullptr, 0, 0, 0, 1, forward_la_kernel<W>, W, false, true}
#define FWD_ROW_VARIANT(K) {"fwd_row_k" #K, 64, K, 0, nullptr, nullptr, 0, 0, 0, 1, nullptr, 0, false, false, forward_row_kernel<K>, K}

const Variant kVariants[] = {
    // The paper's three GPU programs as (rows per lane K, j-unroll U):
    // gpu-no-unrolling (1, 1), simple-unrolling (4, 1) and double-unrolling
    // (4, 4) of Figs. no-u, sim-u and double-u (Sec. IV).
    FWD_VARIANT(256, 1, 1),
    FWD_VARIANT(256, 4, 1),
    FWD_VARIANT(256, 4, 4),
    FWD_VARIANT(256, 2, 8),
    FWD_VARIANT(256, 1, 8),
    FWD_VARIANT(128, 2, 8),
    FWD_VARIANT(128, 1, 8),
    FWD_VARIANT(64, 1, 8),
    FWD_VARIANT(64, 2, 8),
    FWD_VARIANT(64, 4, 4),
    FWD_VARIANT(64, 1, 16),
    FWD_SYM_VARIANT(8, 4, 1),
    FWD_SYM_VARIANT(8, 4, 2),
    FWD_SYM_VARIANT(4, 8, 1),
    FWD_SYM_VARIANT(4, 4, 1),
    FWD_SYM_VARIANT(2, 8, 1),
    FWD_SYM_VARIANT(16, 4, 1),
    FWD_SYM_VARIANT(2, 4, 1),
    FWD_SYM_VARIANT(1, 4, 1),
    FWD_SYM_VARIANT(1, 2, 1),
    FWD_SYM_VARIANT(2, 2, 1),
    FWD_SYM_VARIANT(4, 2, 1),
    FWD_SYM_R_VARIANT(1, 4, 8),
    FWD_SYM_R_VARIANT(1, 2, 8),
    FWD_SYM_R_VARIANT(4, 4, 8),
    FWD_SYM_R_VARIANT(8, 4, 8),
    FWD_LA_VARIANT(4),
    FWD_LA_VARIANT(8),
    FWD_LA_VARIANT(16),
    FWD_LA1_VARIANT(8),
    FWD_LA1_VARIANT(16),
    FWD_ROW_VARIANT(1),
    FWD_ROW_VARIANT(2),
    FWD_ROW_VARIANT(4),
    // float64 running sums, for accuracy at very large n
    FWD_D64_VARIANT(256, 1, 8),
    FWD_D64_VARIANT(64, 1, 8),
    FWD_D64_VARIANT(128, 2, 8),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

int forward_variant_count() { return kNumVariants; }

const char *forward_variant_name(int index)
{
    return (index >= 0 && index < kNumVariants) ? kVariants[index].name : nullptr;
}

static int variant_index(const char *name)
{
    for (int v = 0; v < kNumVariants; ++v)
        if (std::strcmp(kVariants[v].name, name) == 0) return v;
    return 0;
}

// Measured on MI355X: the pair-once kernel wins from about 4,500 particles
// on, one wave per row below.  Its
// workspace is bounded (ring groups, about 1 GiB up to 2^22 particles,
// 256 n bytes above); beyond 2^24 particles, where a group would hold very
// few ring offsets, the float64-sum gather takes over.
int forward_default_variant(int64_t n)
{
    // The gather keeps float64 row sums: as fast as float32 sums and
    // 10-100x more accurate above a million bodies.
    static const int gather_big = variant_index("fwd_b64_k1_u8_f64sum");
    static const int row_1 = variant_index("fwd_row_k1");
    static const int row_2 = variant_index("fwd_row_k2");
    static const int pair_once_8 = variant_index("fwd_sym_w8_k4_r8");
    static const int pair_once_4 = variant_index("fwd_sym_w4_k4_r8");
    static const int pair_once_1 = variant_index("fwd_sym_w1_k4_r8");
    static const int pair_once_1s = variant_index("fwd_sym_w1_k2_r8");
    static const int pair_once_small = variant_index("fwd_sym_w1_k2_o1");
    if (n > (1 << 24)) return gather_big;
    // Eight rounds of workgroups (each block's tiles cut into eight times as
    // many chunks as the device holds workgroups), which the dispatcher
    // hands out as slots free up, also pay at large n, where one round
    // leaves every workgroup a whole ring group of tiles and each launch
    // ends on its slowest: forced-variant sweep, same box, 6.7% less time
    // than one round at 2^20 for 8-wave blocks of 2,048 particles (the
    // same five ring-group launches), and 4-wave blocks of 1,024 in eight
    // rounds 1-7% ahead from 2^17 to 2^19 (up to 15% ahead of the 8-wave
    // ones there).  Below 2^16 likewise 2-8% from 16,384 to 65,536
    // (interleaved A/B in one process).  The 4-wave blocks lead the
    // one-wave four-row ones from 40,000 bodies (1-5% from 40,000 to
    // 60,000, 3-5% behind at 36,000; forced-variant sweep, same box).
    if (n >= (1 << 20)) return pair_once_8;
    if (n >= 40000) return pair_once_4;
    // four-row one-wave blocks lead from about 18,000 (2% at 18,000 and
    // 22,000, 3% at 24,000; 1-2% behind at 16,384)
    if (n >= 18000) return pair_once_1;
    // eight rounds of one-wave blocks of 128 particles from 10,000: below
    // that one round already cuts every block's sequence into one-tile
    // chunks (the same plan, the same time), above it one round leaves
    // chunks of one and two tiles and takes 11% longer (11,000 and 12,000
    // bodies, forced-variant sweep, same box)
    if (n >= 10000) return pair_once_1s;
    // one-wave blocks of 128 particles: twice the workgroups of 256-particle
    // blocks, which evens out the one round of workgroups these sizes fill
    // (3-17% faster from 3,000 to 10,000 bodies)
    // Small n is set by launch latency and the longest dependent chain: one
    // wave per row (two rows from 3,000 bodies), no LDS, no second launch.
    // Kernel 3.4 us at 1,024 bodies against 7.1 us for the one-launch split
    // gather.  Against the pair-once kernel and its fold (forced variants,
    // same box) the row kernel leads up to 4,000 bodies (plain calls 17.3
    // against 20.6 us, leap-frog steps 13.9 against 16.4 us), is level with
    // it for plain calls with the potential at 4,500 and behind from 5,000
    // (22.5 against 22.0 us); a leap-frog step, whose update the pair-once
    // fold applies in place and the row kernel needs a launch for, is 6-14%
    // faster pair-once from 4,500 to 5,000.  Both use one choice, so that a
    // leap-frog call stays bitwise the composed calls.
    if (n >= 4500) return pair_once_small;
    return n >= 3000 ? row_2 : row_1;
}

bool forward_variant_f64sum(int v) { return v >= 0 && v < kNumVariants && kVariants[v].d64; }

int forward_default_f64sum_variant(int64_t n)
{
    static const int big = variant_index("fwd_b64_k1_u8_f64sum");
    static const int mid = variant_index("fwd_b256_k1_u8_f64sum");
    return n > (1 << 17) ? big : mid;
}

// Number of j-splits: enough workgroups to give every CU several, never a
// split smaller than one tile.
static int choose_splits(int n, int iblocks, int tile, int num_cu)
{
    const int target = 4 * num_cu;
    const int max_splits = (n + tile - 1) / tile;
    int s = (target + iblocks - 1) / iblocks;
    if (s < 1) s = 1;
    if (s > max_splits) s = max_splits;
    return s;
}

// Geometry of the one-launch kernel for n rows: j-splits per 64-row block
// and j per wave.  Waves per row block: about 4096 waves over the chip (4
// per SIMD), at least 32 j per wave, at most n / 32 waves.
static void la_geometry(const Variant &V, int n, int num_cu, int *splits_out, int *chunk_out)
{
    const int rb = (n + 63) / 64;
    int per_rb = std::max(1, 4 * 4 * num_cu / rb);
    per_rb = std::min(per_rb, std::max(1, n / 32));
    int splits = V.la_one ? 1 : std::max(1, (per_rb + V.la_w / 2) / V.la_w);
    const int waves = splits * V.la_w;
    int chunk = (n + waves - 1) / waves;
    chunk = chunk >= 64 ? (chunk + 63) / 64 * 64 : (chunk + 15) / 16 * 16;
    splits = std::max(1, (int)(((int64_t)n + (int64_t)chunk * V.la_w - 1) / ((int64_t)chunk * V.la_w)));
    *splits_out = splits;
    *chunk_out = chunk;
}

// Geometry of the row gather: j-splits and j per split (a multiple of the
// tile).
static void gather_geometry(const Variant &V, int n, int num_cu, int *splits_out, int *chunk_out)
{
    const int iblk = V.block * V.k;
    const int iblocks = (n + iblk - 1) / iblk;
    int splits = choose_splits(n, iblocks, V.block, num_cu);
    int chunk = (n + splits - 1) / splits;
    chunk = (chunk + V.block - 1) / V.block * V.block;
    *splits_out = (n + chunk - 1) / chunk;
    *chunk_out = chunk;
}

int64_t forward_plan_bytes(int variant, int64_t n, int num_cu, int per_cu)
{
    if (variant < 0 || variant >= kNumVariants || n < 0 || n > NBODY_MAX_N || num_cu < 1 ||
        per_cu < 1)
        return -1;
    if (n == 0) return 0;
    const Variant &V = kVariants[variant];
    int splits = 1, chunk = 0;
    if (V.row) return 0;
    if (V.la_w) {
        la_geometry(V, (int)n, num_cu, &splits, &chunk);
        return splits > 1 ? (int64_t)sizeof(float4) * splits * n : 0;
    }
    if (V.sym_w) {
        SymPlan pl;
        if (!sym_plan(n, V.sym_w * 64 * V.sym_k, (int64_t)per_cu * num_cu * V.sym_rounds, V.sym_occ,
                      sym_workspace_budget(n), &pl))
            return -1;
        return (int64_t)pl.bytes();
    }
    gather_geometry(V, (int)n, num_cu, &splits, &chunk);
    const int64_t entry = V.d64 ? 4 * (int64_t)sizeof(double) : (int64_t)sizeof(float4);
    return splits > 1 ? entry * splits * n : 0;
}

int64_t forward_variant_max_n(int variant)
{
    if (variant < 0 || variant >= kNumVariants) return -1;
    // the one-launch kernels are built for launch-latency-bound sizes
    return (kVariants[variant].la_w || kVariants[variant].row) ? (1 << 16) : NBODY_MAX_N;
}

nbody_status forward_variant_occupancy(int variant, int *per_cu)
{
    const Variant &V = kVariants[variant];
    hipError_t e;
    if (V.sym_w) return forward_sym_occupancy(V.sym_w, V.sym_k, per_cu);
    if (V.row)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, V.row, 256, 0);
    else if (V.la_w)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, V.la, V.la_w * 64, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, V.partial, V.block, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (*per_cu < 1) *per_cu = 1;
    return NBODY_OK;
}

nbody_status forward_run(int variant, const Device &dev, const float *x, const float *m, int n,
                         float eps2, float *a, float *p, hipStream_t stream, const LfEpi *epi,
                         bool *fused, const Arena &arena)
{
    const Variant &V = kVariants[variant];
    if (fused) *fused = false;
    if (V.row) {
        const int64_t waves = ((int64_t)n + V.row_k - 1) / V.row_k;
        RowArgs P{x, m, n, eps2, a, p};
        if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
        prof_mark(stream, 0);
        hipLaunchKernelGGL(V.row, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, stream, P);
        prof_mark(stream, 1);
        return check_launch(V.name);
    }
    if (V.la_w) {
        const int rb = (n + 63) / 64;
        int splits = 1, chunk = 0;
        la_geometry(V, n, dev.num_cu, &splits, &chunk);
        LaArgs P{x, m, n, eps2, chunk, splits, nullptr, nullptr, a, p};
        if (splits > 1) {
            void *ws = nullptr;
            nbody_status st = arena.get(dev, stream, sizeof(float4) * (size_t)splits * n, &ws);
            if (st != NBODY_OK) return st;
            P.partial = static_cast<float4 *>(ws);
            st = arena.get_counters(dev, stream, (size_t)rb, &P.ctr);
            if (st != NBODY_OK) return st;
        }
        if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
        prof_mark(stream, 0);
        hipLaunchKernelGGL(V.la, dim3(rb, splits), dim3(V.la_w * 64), 0, stream, P);
        prof_mark(stream, 1);
        return check_launch(V.name);
    }
    if (V.sym_w)
        return forward_sym_run(V.sym_w, V.sym_k, V.sym_occ, V.sym_rounds, V.name, dev, x, m, n, eps2,
                               a, p, stream, epi, fused, arena);
    const int iblk = V.block * V.k;
    const int iblocks = (n + iblk - 1) / iblk;
    int splits = 1, chunk = 0;
    gather_geometry(V, n, dev.num_cu, &splits, &chunk);

    FwdArgs P{x, m, n, eps2, chunk, nullptr, a, p, nullptr};
    if (splits == 1) {
        if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
        prof_mark(stream, 0);
        hipLaunchKernelGGL(V.direct, dim3(iblocks, 1), dim3(V.block), 0, stream, P);
        prof_mark(stream, 1);
        return check_launch(V.name);
    }
    void *ws = nullptr;
    const size_t entry = V.d64 ? 4 * sizeof(double) : sizeof(float4);
    nbody_status st = arena.get(dev, stream, entry * (size_t)splits * n, &ws);
    if (st != NBODY_OK) return st;
    if (V.d64)
        P.partial_d = static_cast<double *>(ws);
    else
        P.partial = static_cast<float4 *>(ws);
    if (fault_injected("launch")) return fail(NBODY_ERROR_LAUNCH_FAILED, "injected launch fault");
    prof_mark(stream, 0);
    hipLaunchKernelGGL(V.partial, dim3(iblocks, splits), dim3(V.block), 0, stream, P);
    prof_mark(stream, 1);
    st = check_launch(V.name);
    if (st != NBODY_OK) return st;
    if (V.d64)
        hipLaunchKernelGGL(reduce_splits_d_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                           P.partial_d, splits, n, a, p);
    else
        hipLaunchKernelGGL(reduce_splits_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                           P.partial, splits, n, a, p);
    return check_launch("reduce_splits");
}

}  // namespace nbody
