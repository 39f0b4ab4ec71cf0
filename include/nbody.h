/*
 * nbody.h -- C ABI of libnbody.so: the exact softened all-pairs gravity sum
 * of Fujiwara & Nakasato, "Fast Simulations of Gravitational Many-body
 * Problem on RV770 GPU" (arXiv:0904.3659), on AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays are device pointers (memory of the current HIP device), float32,
 *   row-major, densely packed: positions x[n][3], masses m[n], accelerations
 *   a[n][3], potentials p[n].  The caller owns every array; the library never
 *   frees or retains caller memory beyond the call.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *   is asynchronous with respect to the host and ordered on `stream`; faults
 *   inside a kernel surface at the caller's next synchronisation.
 * - Outputs are fully overwritten, never accumulated into, except the
 *   in/out arrays of the element-wise and leap-frog calls (stated there).
 *   Inputs and outputs must not overlap (checked on the host from the
 *   address ranges).
 * - Library workspace (partial sums, work lists) is device memory owned by
 *   the library, cached per (device, stream) and grown on demand; it is held
 *   until nbody_release_workspace() or process exit.  Calls that share one
 *   stream reuse it safely; calls on different streams use different
 *   workspaces.
 * - HIP graph capture: nbody_forces, nbody_forces_ex, nbody_forces_backward,
 *   nbody_forces_batched, nbody_axpy, nbody_kick_drift, nbody_leapfrog and
 *   nbody_leapfrog_adjoint may be captured on a stream once the same call
 *   has run eagerly on that stream (so that the
 *   stream's workspace, counters and the batched plan exist; a first call
 *   allocates and a first batched call synchronises, which capture forbids).
 *   The graph keeps the workspace addresses of that stream (partial sums,
 *   the leap-frog adjoint's 16 n-byte buffer, counters): while it may
 *   replay, make no call on that stream that needs a larger one of them, do
 *   not call nbody_release_workspace(), run no variant timer
 *   (nbody_autotune, nbody_autotune_batched) on that stream, and keep the
 *   number of distinct (offsets, variant) pairs of batched
 *   calls below the plan cache size (8).  No memset is recorded: counters
 *   are cleared by the kernels that use them.
 * - No C++ exception crosses this interface.  Every call returns a status;
 *   on failure nbody_last_error() gives a thread-local detail string.
 *   Argument checks run before any HIP call, so an invalid call touches no
 *   device state.
 * - n is limited to NBODY_MAX_N particles (per system for the batched call,
 *   and in total).
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBODY_ABI_VERSION 4
#define NBODY_MAX_N (INT64_C(1) << 28)
#define NBODY_MAX_STEPS (INT64_C(1) << 30)

typedef enum nbody_status {
    NBODY_OK = 0,
    NBODY_ERROR_INVALID_ARGUMENT = 1,   /* bad size, pointer, eps2, offsets, overlap */
    NBODY_ERROR_UNSUPPORTED_DEVICE = 2, /* current device is not gfx950 */
    NBODY_ERROR_OUT_OF_MEMORY = 3,      /* workspace allocation failed */
    NBODY_ERROR_LAUNCH_FAILED = 4,      /* a kernel launch was rejected */
    NBODY_ERROR_INTERNAL = 5            /* any other HIP runtime error */
} nbody_status;

/* Kinds of evaluation, for variant selection and tuning. */
typedef enum nbody_kind {
    NBODY_KIND_FORWARD = 0,
    NBODY_KIND_BACKWARD = 1,
    NBODY_KIND_BATCHED = 2
} nbody_kind;

/* NBODY_ABI_VERSION of the built library. */
int nbody_abi_version(void);

/* Static, never-NULL name of a status code. */
const char *nbody_status_string(nbody_status status);

/* Thread-local detail of the last failed call on this thread ("" if none). */
const char *nbody_last_error(void);

/*
 * Forward evaluation, Eq. (gravity) of Sec. I, in the paper's sign:
 *     a_i = sum_{j != i} m_j (x_i - x_j) / (|x_i - x_j|^2 + eps2)^(3/2)
 *     p_i = sum_{j != i} m_j / (|x_i - x_j|^2 + eps2)^(1/2)
 * (a points from x_j towards x_i, p is positive; the physical acceleration
 * is -a).  G = 1.  The term j == i is excluded by index, so no self
 * potential m_i/eps appears.  One softening eps2 = eps^2 serves every pair.
 *
 * x: [n][3] in, m: [n] in, a: [n][3] out, p: [n] out (p may be NULL to skip
 * the potential; the pair-once kernels then do not form its terms, and a is
 * bitwise the same as with p).
 * Arithmetic: float32 with fused multiply-add, hardware reciprocal square
 * root, and partial sums folded per j-tile (two-level accumulation).
 * The result is bitwise reproducible for a fixed n, variant and device.
 * Kernels: for 4,500 <= n <= 2^24 the default variant evaluates each
 * unordered pair once and gives the term to both particles (the softened
 * force is antisymmetric in the pair), in blocks of P = 2048 particles from
 * 2^20 up, 1024 from 40,000, 256 from 18,000 and 128 below.  Each block meets
 * the blocks after it on a ring; the ring offsets run in groups, one launch
 * per group, each followed by a launch that adds the group's partial sums
 * to a float64 running sum per particle, so the library workspace stays at
 * most 1 GiB up to n = 2^22 (256 n bytes above; 0.97 GiB at n = 2^20).
 * Outside that range the default evaluates every ordered pair: below 4,500
 * in one launch with one wave per row (two rows from 3,000), its lanes
 * splitting j and their sums added by a fixed in-register butterfly (no
 * workspace); above 2^24 gathered per row with j-splits, float64 row sums
 * (as NBODY_FORCES_F64_SUM below) and a reduction launch (at most
 * 32 n * splits bytes).
 * Positions must be finite with magnitude below 1e17 (padding slots sit
 * at +-1e18 with zero mass).
 *
 * Errors: n < 0 or n > NBODY_MAX_N, NULL x/m/a with n > 0, eps2 negative or
 * not finite, overlapping arrays -> INVALID_ARGUMENT.  n == 0 -> OK, nothing
 * launched.  n == 1 -> a = 0, p = 0.  eps2 == 0 is allowed; then two distinct
 * particles at the same position give inf/NaN (IEEE), not an error.  NaN or
 * inf inside x or m is not checked and propagates.
 */
nbody_status nbody_forces(const float *x, const float *m, int64_t n, float eps2,
                          float *a, float *p, void *stream);

/* Bytes of device memory behind nbody_forces_noalloc, per device. */
#define NBODY_NOALLOC_SCRATCH_BYTES (INT64_C(64) << 20)

/*
 * nbody_forces for callers that cannot allocate device memory: code under
 * HIP graph capture, serving loops that must not call hipMalloc, harnesses
 * that forbid it.  Same sum, arguments, layouts, ownership, variant choice
 * and errors as nbody_forces, and bitwise its result whenever that call's
 * workspace would fit the region below (or NBODY_SYM_WORKSPACE holds
 * nbody_forces to the region's NBODY_NOALLOC_SCRATCH_BYTES - 4096 bytes);
 * where it would not, the ring runs in more launches and the two results
 * differ in rounding only.  The call itself allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).
 *
 * Its workspace is a fixed region of NBODY_NOALLOC_SCRATCH_BYTES (64 MiB)
 * of device memory that the library holds on every device it runs on until
 * the process ends (its last 4 KiB are int counters, zeroed by a fill
 * kernel on `stream` at the first call on a device).  The pair-once kernels
 * split their ring into more launches to fit it, which bounds n at about
 * 2^20 particles; a call whose kernels cannot fit the region returns
 * INVALID_ARGUMENT with the sizes in nbody_last_error().
 * Every call on one device shares that device's region and leaves the last
 * call's partial sums in it: calls that overlap in time on one device (two
 * streams, two host threads) race and give undefined results.  Serialise
 * them, or use nbody_forces.
 */
nbody_status nbody_forces_noalloc(const float *x, const float *m, int64_t n, float eps2,
                                  float *a, float *p, void *stream);

/* Flag bits of nbody_forces_ex. */
#define NBODY_FORCES_F64_SUM 1u

/*
 * nbody_forces with option flags; nbody_forces(...) is
 * nbody_forces_ex(..., 0u, stream).  Same sum, arguments, layouts, ownership
 * and errors as nbody_forces.
 *
 * NBODY_FORCES_F64_SUM: keep each row's running sum in float64.  The pair
 * terms and each j-tile's sum (64 to 256 terms) stay float32; the tile
 * sums, and the j-split partials, are added in float64 and rounded to
 * float32 once at the store.  Float32 running sums add n / tile tile sums in
 * float32, an error that grows with n; the paper computes in single
 * precision throughout (Sec. IV).  The default pair-once kernel adds its
 * partial sums in float64 across ring groups, and above 2^24 the default
 * sums in float64 as this flag does; the flag trades the pair-once (or
 * one-launch) kernel for the row gather (about 30% slower at n = 2^20) and
 * 32 n * splits bytes of workspace.  A forced variant (nbody_set_variant)
 * is honoured only if it is one of the "_f64sum" variants.
 * Errors: as nbody_forces; unknown flag bits -> INVALID_ARGUMENT.
 */
nbody_status nbody_forces_ex(const float *x, const float *m, int64_t n, float eps2,
                             float *a, float *p, uint32_t flags, void *stream);

/*
 * Backward (vector-Jacobian product) of nbody_forces, derived from
 * Eq. (gravity) by the chain rule.  For upstream gradients grad_a = dL/da
 * [n][3] and grad_p = dL/dp [n], with d = x_k - x_j, s = |d|^2 + eps2,
 * r = s^(-1/2), c_kj = m_j grad_a_k - m_k grad_a_j,
 * b_kj = m_j grad_p_k + m_k grad_p_j:
 *     grad_x_k = sum_{j != k} r^3 [ c_kj - (3 r^2 (c_kj . d) + b_kj) d ]
 *     grad_m_k = sum_{j != k} r [ grad_p_j - r^2 (grad_a_j . d) ]
 *
 * grad_a or grad_p may be NULL (meaning zero).  grad_m may be NULL (skip).
 * grad_x: [n][3] out, grad_m: [n] out.  Same arithmetic, determinism and
 * error rules as nbody_forces; NULL grad_x with n > 0 -> INVALID_ARGUMENT.
 * Kernels: for 4,000 <= n <= 2^24 the default variant evaluates each
 * unordered pair once (the x-gradient term is antisymmetric in the pair),
 * for blocks of P = 1024 particles from 2^18, 512 from 40,000 and 128
 * below (from 4,000 to 11,999 two waves share a block's rows and split
 * each tile's steps), with the ring groups and bounded workspace of the
 * pair-once forward (at most 1 GiB up to n = 2^22).  With grad_p NULL it
 * does not form the potential-weight terms (with the same variant, bitwise
 * the result of zero weights); the default variant is the same.  Below 4,000 one
 * launch with one wave per row (two rows from 3,500) evaluates every
 * ordered pair (no workspace); above 2^24 every ordered pair is gathered
 * per row.
 */
nbody_status nbody_forces_backward(const float *x, const float *m, int64_t n, float eps2,
                                   const float *grad_a, const float *grad_p,
                                   float *grad_x, float *grad_m, void *stream);

/*
 * Eq. (gravity) on many independent systems in one launch.  System s owns
 * particles [offsets[s], offsets[s+1]) of x, m, a, p and interacts only with
 * itself.  `offsets` is a HOST array of num_systems + 1 int64 values with
 * offsets[0] == 0, non-decreasing; the total is offsets[num_systems].
 * Empty systems are allowed.  The library builds a work plan from the
 * offsets (a cost-ordered list of units: (system, 256-particle block) for
 * the default pair-once variant, (system, i-tile) for gather variants),
 * caches it keyed by the offsets' content, uploads it to library memory and
 * runs one persistent launch whose workgroups draw units largest-first from
 * a per-stream ticket counter (plus one launch that adds the pair-once
 * partial sums; about 16 (1 + M_s/2) N_s bytes of workspace per system of
 * N_s particles in M_s blocks).  Per-system results equal nbody_forces on
 * that system up to float32 summation order, and are bitwise independent of
 * the other systems' contents.
 *
 * Errors: num_systems < 0, NULL offsets, offsets[0] != 0, a decreasing
 * offset, a system or the total above NBODY_MAX_N -> INVALID_ARGUMENT; plus
 * the pointer, eps2 and overlap rules of nbody_forces.
 */
nbody_status nbody_forces_batched(const int64_t *offsets, int64_t num_systems,
                                  const float *x, const float *m, float eps2,
                                  float *a, float *p, void *stream);

/*
 * Leap-frog kick and drift (Eqs. (1)-(3) of Sec. III) as device kernels, so
 * an integrator can stay on the device between force evaluations:
 *     nbody_axpy:  y[t] += alpha * xv[t]   for t < len   (float32 FMA)
 * A kick with the paper's a is nbody_axpy(v, a, -dt/2) (the physical
 * acceleration is -a); a drift is nbody_axpy(x, v, dt).
 * Errors: len < 0, NULL with len > 0, alpha not finite, overlap ->
 * INVALID_ARGUMENT.
 */
nbody_status nbody_axpy(float *y, const float *xv, int64_t len, float alpha, void *stream);

/*
 * Kick and drift of one leap-frog step in one pass (Eqs. (1)-(2), Sec. III):
 *     v += kick * a;  x += dt * v        (x, v, a: [n][3], float32 FMA)
 * With the paper's a, kick = -dt/2 (the physical acceleration is -a).
 * Errors: n < 0 or > NBODY_MAX_N, NULL with n > 0, kick or dt not finite,
 * overlapping arrays -> INVALID_ARGUMENT.
 */
nbody_status nbody_kick_drift(float *x, float *v, const float *a, int64_t n, float kick, float dt,
                              void *stream);

/*
 * `steps` leap-frog (kick-drift-kick) steps on the device, Eqs. (1)-(3) of
 * Sec. III with the physical acceleration -a (a in the paper's sign, as
 * nbody_forces gives it) and no potential:
 *     repeat steps times:  v += -dt/2 a;  x += dt v;  a = a(x);  v += -dt/2 a
 * x, v: [n][3] in/out.  a: [n][3] in/out: a(x) on entry (nbody_forces with
 * the same n and eps2), a of the final positions on exit.  m: [n] in.
 * x_hist: NULL, or [steps][n][3] out: x_hist[t] receives the positions
 * after step t + 1 (x_hist[steps - 1] equals x on exit).
 * The result is bitwise that of the call sequence
 *     nbody_kick_drift(x, v, a, n, -dt/2, dt);
 *     nbody_forces(x, m, n, eps2, a, NULL);
 *     nbody_axpy(v, a, 3 n, -dt/2);
 * repeated steps times (the same float32 FMAs in the same order).  A
 * step's end kick, the next step's start kick and its drift run in the
 * final reduction kernel of the pair-once force variants (two launches per
 * step), otherwise in one element-wise launch after the force.  Library
 * memory: that of nbody_forces.
 * Errors: n < 0 or > NBODY_MAX_N, steps < 0 or > NBODY_MAX_STEPS, eps2 as
 * for nbody_forces, dt not finite, NULL x, v, a or m with n > 0 and
 * steps > 0, any two of x, v, a, m, x_hist overlapping -> INVALID_ARGUMENT.
 */
nbody_status nbody_leapfrog(float *x, float *v, float *a, const float *m, int64_t n, float eps2,
                            float dt, int64_t steps, float *x_hist, void *stream);

/* Flags of nbody_leapfrog_adjoint. */
#define NBODY_LEAPFROG_FINAL 1u   /* the segment ends at the final state */
#define NBODY_LEAPFROG_INITIAL 2u /* the segment starts at the initial state */

/*
 * Reverse sweep over one segment of `steps` nbody_leapfrog steps: the
 * vector-Jacobian product of the steps with respect to the positions,
 * velocities and masses (the adjoint of a checkpointed integration, one
 * segment per call, last segment first).
 * pos: [steps + 1][n][3] in, the positions the forward pass visited:
 *   pos[0] at the segment's start, pos[t] after its t-th step.
 * lx, lv: [n][3] in/out: dL/dx and dL/dv at the segment's end on entry,
 *   at its start on exit.  lm: [n] in/out: dL/dm, accumulated (+=).
 * Each kick is a VJP of Eq. (gravity) with weights lv on a
 * (nbody_forces_backward with grad_a = lv, grad_p = NULL) added to lx and
 * lm with the factor c of its kicks: at pos[t], 1 <= t < steps, the end
 * kick of step t and the start kick of step t + 1 (c = -dt); at pos[0] the
 * first start kick plus, without NBODY_LEAPFROG_INITIAL, the end kick of
 * the step before the segment (c = -dt/2 with the flag, else -dt); at
 * pos[steps] the last end kick, only with NBODY_LEAPFROG_FINAL (c = -dt/2;
 * without the flag the next segment's sweep has covered it).  Order, from
 * the segment's end: [final end kick,] then per step t = steps..1:
 *     lv += dt lx;  lx += c VJP(pos[t-1])[lv];  lm += c VJP_m(pos[t-1])[lv]
 * bitwise as that sequence of nbody_axpy and nbody_forces_backward calls.
 * The updates run in the final reduction kernel of the pair-once adjoint
 * variants (the next step's lv += dt lx with them).  Library memory: that
 * of nbody_forces_backward plus 16 n bytes per (device, stream).
 * Errors: unknown flag bits, n, steps, eps2 or dt as for nbody_leapfrog,
 * NULL pos, m, lx, lv or lm with n > 0 and steps > 0, any two arrays
 * overlapping -> INVALID_ARGUMENT.
 */
nbody_status nbody_leapfrog_adjoint(const float *pos, const float *m, int64_t n, float eps2,
                                    float dt, int64_t steps, uint32_t flags, float *lx, float *lv,
                                    float *lm, void *stream);

/* ---------------------------------------------------------------- tuning */

/* Number of compiled kernel variants for a kind (0 for an unknown kind). */
int nbody_variant_count(int kind);

/* Static name of variant `index` of `kind` (NULL if out of range). */
const char *nbody_variant_name(int kind, int index);

/*
 * Force variant `index` for `kind` on this process (-1 restores automatic
 * choice).  The environment variable NBODY_VARIANT=<kind>:<index>[,...]
 * sets the same at load time.  Out-of-range index -> INVALID_ARGUMENT.
 */
nbody_status nbody_set_variant(int kind, int index);

/*
 * Time every variant of `kind` on each size in sizes[count] (synthetic
 * inputs in library workspace, HIP events on `stream`) and record the
 * fastest per size bucket in the in-process tuning table; if the
 * environment variable NBODY_TUNE_CACHE names a file, the table is also
 * written there as JSON and read back at load time.  Blocks the host until
 * the timing runs finish.  For NBODY_KIND_BATCHED each size is the number of
 * particles per system of a uniform ensemble holding about 2^22 particles.
 */
nbody_status nbody_autotune(int kind, const int64_t *sizes, int64_t count, void *stream);

/*
 * The variant timer on the caller's own ensemble: time every batched
 * variant on (offsets, x, m, eps2) exactly as nbody_forces_batched would
 * run it (results go to library-allocated scratch arrays, freed before
 * returning) and record the fastest for the bucket of the mean system size
 * offsets[num_systems] / num_systems, as nbody_autotune does.  Blocks the
 * host until the timing runs finish.  The timing runs build their plans
 * outside the plan cache and free them; only the winner's plan is then
 * built into the cache (one ordinary run).  The runs use `stream` and may
 * grow its workspace.
 * Errors: the offsets, eps2, pointer and overlap rules of
 * nbody_forces_batched -> INVALID_ARGUMENT; OUT_OF_MEMORY if the scratch
 * arrays cannot be allocated.
 */
nbody_status nbody_autotune_batched(const int64_t *offsets, int64_t num_systems, const float *x,
                                    const float *m, float eps2, void *stream);

/*
 * The launch plan of variant `index` of NBODY_KIND_FORWARD or
 * NBODY_KIND_BACKWARD at size n, computed on the host from the arguments
 * alone (no device is touched): returns the bytes of library workspace one
 * call needs on a device of num_cu compute units where the variant's pair
 * kernel fits blocks_per_cu workgroups per CU, and sets *timed (if not NULL)
 * to whether nbody_autotune would time the variant there with free_bytes
 * of free device memory.  The timer times a variant only if n lies in its
 * size band (the one-launch forward kernels stop at 2^16) and its workspace
 * fits the smaller of NBODY_TUNE_WORKSPACE_CAP bytes (environment; default
 * 2 GiB) and a quarter of the free memory; a variant whose allocation fails
 * while timing is skipped as well, and the workspace the timing grew on the
 * stream is given back when it ends.  The pair-once variants bound their
 * workspace by running their ring of block offsets in several launches: at
 * most 1 GiB (or 256 n bytes where n > 2^22).
 * Returns -1 for an unknown kind or index, n outside [0, NBODY_MAX_N],
 * num_cu or blocks_per_cu below 1, free_bytes below 0.
 */
int64_t nbody_variant_plan(int kind, int index, int64_t n, int num_cu, int blocks_per_cu,
                           int64_t free_bytes, int *timed);

/*
 * Variant index the library would use for `kind` at size n (-1 on error);
 * for NBODY_KIND_BACKWARD the same with and without grad_p and in
 * nbody_leapfrog_adjoint.
 */
int nbody_selected_variant(int kind, int64_t n);

/* Free every cached workspace of every device and stream (synchronises). */
nbody_status nbody_release_workspace(void);

/* -------------------------------------------------------------- profiling */

/*
 * Kernel timing of the library's own launches.  While enabled (on != 0),
 * every successful nbody_forces / nbody_forces_backward /
 * nbody_forces_batched call (and each step of nbody_leapfrog and
 * nbody_leapfrog_adjoint) of the calling thread records HIP events on its
 * stream: before and after each of its pair kernels (a pair-once call
 * launches one per ring group) and after its last kernel (the partial-sum
 * fold, if any).  The last 256 calls are kept.  Enabling or disabling
 * clears the record.  Costs two event records per pair kernel and one per
 * call; off by default.
 */
nbody_status nbody_profile_enable(int on);

/*
 * Wait for the recorded calls of this thread and return the mean over them
 * of the summed durations of a call's pair kernels (main_ms), of the time
 * from its first pair kernel's start to its last kernel's end (total_ms)
 * and of the number of pair kernels a call launched (launches), and their
 * number (calls; 0 leaves the means at 0).  Clears the record.  NULL
 * outputs are skipped.
 */
nbody_status nbody_profile_read(double *main_ms, double *total_ms, int *calls, double *launches);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
