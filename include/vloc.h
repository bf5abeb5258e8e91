/*
 * vloc.h -- C ABI of libvloc: the local-potential action V_loc|psi> on a batch
 * of plane-wave wave functions, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Gao, Mo, Fang, Wang, "Parallel 3-dim fast Fourier transforms with
 * load balancing of the plane waves" (arXiv:1601.07378).
 *   - Plane-wave expansion and its sign: Sec. 2, eq. 2.
 *   - Cutoff sphere: Sec. 2, eq. 3.
 *   - The operator (to real space, multiply by the diagonal V, back): Sec. 2,
 *     the paragraph after eq. 3.
 *   - Compact 3-D FFT (first pass only on columns meeting the sphere, second
 *     only on columns meeting that cylinder, third on the whole cube): Sec. 4.3.
 *   - Greedy distribution of columns by plane-wave count: Sec. 3.2.
 *
 * For each band n and each g = (h, k, l) of the sphere S:
 *   psi_n(j)  = sum_{g in S} c_n(g) exp(-2 pi i (h j1/N1 + k j2/N2 + l j3/N3))
 *   out_n(g)  = (1/N) sum_j exp(+2 pi i (h j1/N1 + k j2/N2 + l j3/N3)) V(j) psi_n(j)
 * with N = N1 N2 N3 and j over the whole grid.
 *   S = { g in Z^3 : |k+G|^2 <= 2 Ecut (1 + 1e-12) },  G = h b1 + k b2 + l b3,
 *   b = 2 pi A^{-T} where the rows of A are the cell vectors a1, a2, a3.
 * The cutoff is read as non-strict with a relative slack of 1e-12 (eq. 3 prints
 * a strict inequality; on integer-radius spheres the shell is then kept).
 * k enters only through S: V is lattice periodic, so exp(-i k.r) cancels
 * between the two transforms and the grids hold the periodic part.
 *
 * Layouts (all contiguous, interleaved complex = {re, im}):
 *   c, out : [nbands][npw] complex, in the plan's canonical G order
 *            (lexicographic on signed (h, k, l); see vloc_plan_gvectors).
 *   V      : [N3][N2][N1] real, x (j1) fastest.
 *   psi_r  : [nbands][N3][N2][N1] complex (diagnostic transforms only).
 * Element type follows the plan's precision: double / double-complex for
 * VLOC_F64, float / float-complex for VLOC_F32.  All data pointers passed to
 * vloc_apply, vloc_g2r and vloc_r2g are DEVICE pointers, at least 16-byte
 * (F64) or 8-byte (F32) aligned; the caller owns them.
 *
 * Every call returns a vloc_status; nothing throws or aborts.  Detail of the
 * last failure on the calling thread: vloc_last_error().
 */
#ifndef VLOC_H
#define VLOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vloc_plan_s *vloc_plan; /* opaque; owned by the library */

typedef enum {
    VLOC_OK = 0,
    VLOC_E_INVALID = -1, /* NULL pointer, negative count, bad option            */
    VLOC_E_GRID = -2,    /* N_i < 1, N_i > 960, a prime factor other than 2, 3,  */
                         /* 5, or one z-plane's occupied part too large for the  */
                         /* plane kernel's 160 KiB of LDS                        */
    VLOC_E_CELL = -3,    /* det(cell) <= 0 or non-finite cell                    */
    VLOC_E_SPHERE = -4,  /* empty sphere, bad Ecut/k, or the sphere's extent on  */
                         /* some axis is >= N_i (two points alias on the grid)  */
    VLOC_E_ALIAS = -5,   /* out overlaps c or V                                 */
    VLOC_E_NOMEM = -6,   /* host or device allocation failed                    */
    VLOC_E_DEVICE = -7   /* HIP runtime error (no device, launch failure, ...)  */
} vloc_status;

typedef enum { VLOC_F64 = 0, VLOC_F32 = 1 } vloc_precision;

/* Deal of z-sticks (columns meeting the sphere) to stick groups; each group is
 * one workgroup of the two stick-transform kernels.  GREEDY is the paper's
 * rule (sort by descending plane-wave count, ties in canonical order, deal in
 * turn; Sec. 3.2); SNAKE reverses every other pass; CONTIGUOUS cuts the
 * canonical order into consecutive runs; UNSORTED deals the canonical order in
 * turn without sorting (the baseline the paper's balancing improves on). */
typedef enum {
    VLOC_DEAL_GREEDY = 0,
    VLOC_DEAL_SNAKE = 1,
    VLOC_DEAL_CONTIGUOUS = 2,
    VLOC_DEAL_UNSORTED = 3
} vloc_deal;

/* Zero-initialised options mean: F64, greedy deal, automatic sizes. */
typedef struct {
    int32_t precision;        /* vloc_precision                                    */
    int32_t deal;             /* vloc_deal                                         */
    int32_t sticks_per_group; /* 0 = automatic; else 1..64                         */
    int32_t band_chunk;       /* most bands (band pairs in the real mode) per launch;
                                 a call is cut into equal chunks of at most this
                                 many; 0 = automatic (stick buffer <= 256 MiB, and
                                 <= 176 MiB in the density passes, whose FP64
                                 partial planes share the last-level cache)       */
    int32_t plane_rows;       /* rows per x-pass batch of one wavefront in the plane
                                 kernel (plane_xmode 1), rows per part N2 / P
                                 (plane_xmode 6); 0 = automatic                    */
    int32_t plane_threads;    /* threads per plane workgroup (64..512, multiple of
                                 64; FP64 plans up to 1024); 0 = automatic (the
                                 planner's choices include 1024 for the FP64 whole
                                 plane, 768 for the FP64 parted plane and 1024 for
                                 the FP32 parted plane).  The density kernels may
                                 run fewer, to hold a work item's density sums in
                                 registers: 512 for the FP64 parted plane with x
                                 split 8 x 16, y split 16 x 8 and two parts (when
                                 plane_threads >= 512); where the FP32 whole
                                 plane leaves one workgroup per CU (more than
                                 80 KiB of LDS), the application runs 1024, and
                                 so do the density kernels of the compiled 128^2
                                 planes (when plane_threads >= 512)              */
    int32_t plane_xwaves;     /* wavefronts of the plane workgroup that run the x
                                 pass (each with its own row buffer); 0 = auto     */
    int32_t plane_xmode;      /* layout of the plane kernel: 0 = automatic (3 where
                                 the whole plane fits in LDS, else 6, else 1); 1 = the
                                 occupied x-planes plus per-wavefront row buffers;
                                 2 = occupied x-planes, one lane quad per x row
                                 (needs N1 in {24, 72, 80, 96} with the matching y
                                 split and N2 <= 128); 3 = the whole plane, x pass
                                 in place over the workgroup (N1 (N2 + 1) elements
                                 <= 160 KiB); 4 = as 3 with the x rows owned by
                                 wavefronts (no workgroup barrier inside the x
                                 pass); 5 = the whole plane in row blocks (FP64,
                                 768 threads, N1 and N2 = 8 L1: one wavefront
                                 runs y stage B to y stage B' of eight rows; two
                                 workgroup barriers per plane); 6 = the parted
                                 plane: the occupied x-planes for the y pass, the
                                 x pass in P parts of N2 / P rows (P dividing L1y;
                                 nxo L1y / P <= plane_threads) through one row
                                 buffer, the other parts in a device scratch of
                                 nxo N2 values per resident workgroup, allocated
                                 with the plan's tables; unless split[1] is given
                                 the longer y codelet comes first                 */
    int32_t split[3];         /* first codelet length L1 of the L = L1 * L2 split of
                                 each axis (x, y, z); 0 = automatic (the most
                                 balanced split); else L1 and L / L1 must both be
                                 codelet lengths {1..6, 8, 9, 10, 12, 15, 16, 18,
                                 20, 24, 25, 27, 30, 32} (x and y codelets above 16
                                 need plane_threads <= 512).
                                 Common grids run kernels compiled for their
                                 automatic split; other splits run the same
                                 kernels with run-time sizes                       */
    int32_t gamma;            /* 1 = real mode (needs k = 0): wave functions are real
                                 in space, c(-g) = conj(c(g)); c and out hold only
                                 the half sphere H = {h > 0} u {h = 0, k > 0} u
                                 {h = k = 0, l >= 0} (canonical order restricted to
                                 H; vloc_plan_npw / gvectors describe H) and two
                                 bands share one complex transform (the paper's
                                 gamma-point variant, Sec. 4.3).  Im c(0) is taken
                                 as 0 and Im out(0) is 0.  Only vloc_apply accepts
                                 such plans                                       */
} vloc_options;

/* Build a plan (host work only; device tables are uploaded on first use).
 *   grid : {N1, N2, N3}, each in [1, 960] with no prime factor other than 2,
 *          3 and 5 (the FFT grids of a plane-wave code, Sec. 2: every such
 *          length splits into two register codelets of at most 32 points).
 *          One z-plane's occupied part, nxo (N2 + 1) complex values plus one
 *          row buffer, must fit in 160 KiB of LDS (else VLOC_E_GRID).
 *   cell : rows a1, a2, a3 (bohr), det > 0.
 *   ecut : Hartree; the sphere keeps |k+G|^2 <= 2 ecut (1 + 1e-12).
 *   k    : reduced coordinates in the reciprocal basis b1, b2, b3.
 * Errors: VLOC_E_INVALID (NULL), VLOC_E_GRID, VLOC_E_CELL, VLOC_E_SPHERE,
 * VLOC_E_NOMEM.  On error *plan is set to NULL. */
vloc_status vloc_plan_create(vloc_plan *plan, const int32_t grid[3], const double cell[9],
                             double ecut, const double k[3]);
/* As vloc_plan_create, with options (NULL = defaults). */
vloc_status vloc_plan_create_ex(vloc_plan *plan, const int32_t grid[3], const double cell[9],
                                double ecut, const double k[3], const vloc_options *opt);
/* Frees host and device resources; NULL is a no-op.  Waits for the plan's
 * stream before freeing device memory. */
vloc_status vloc_plan_destroy(vloc_plan plan);

/* Stream on which the plan enqueues work (a hipStream_t; NULL = the null
 * stream).  The plan does not own the stream.  The plan's stick buffer is
 * reused by every call, so on a change of stream the new stream first waits
 * (hipStreamWaitEvent) for the work already enqueued on the old one. */
vloc_status vloc_set_stream(vloc_plan plan, void *hip_stream);

/* out[n] = V_loc c[n] for n < nbands (definition above).  Stream-ordered and
 * asynchronous: returns after enqueueing.  nbands == 0 is a no-op that returns
 * VLOC_OK.  out must not overlap c or V (VLOC_E_ALIAS); c and V are not
 * modified.  The plan owns an internal stick buffer sized for one band chunk,
 * allocated on first use; calls on one plan must not run concurrently. */
vloc_status vloc_apply(vloc_plan plan, const void *c, int64_t nbands, const void *V, void *out);

/* Allocation-free variant of vloc_apply, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, result and stream ordering as
 * vloc_apply (bitwise the same output), but the kernels' scratch (the
 * potential in the plane kernel's order and the stick buffer) lives in one
 * static device array of 64 MiB per GPU, held until the process ends, and the
 * call makes no hipMalloc, hipFree or other allocation.  Preconditions, each
 * refused with VLOC_E_INVALID and a message: the plan's tables are already on
 * the device (its first vloc_apply call uploads them), the current device is
 * the plan's, and one band fits: N1 N2 N3 real values (whole-plane layouts)
 * plus N3 nsticks complex values at most 64 MiB (bands then run in chunks of
 * as many as fit).  The scratch needs no clearing (every call writes all of
 * it before reading it).  Every call on one GPU shares that GPU's array, from
 * any plan: calls that overlap on one GPU (other streams, other threads)
 * race and give wrong results; order them on one stream.  Timing
 * (vloc_plan_enable_timing) is not recorded on this path. */
vloc_status vloc_apply_noalloc(vloc_plan plan, const void *c, int64_t nbands, const void *V,
                               void *out);

/* ---------------------------------------------------------------- queries */
/* Host outputs, caller-allocated.  npw and gvectors describe the
 * coefficients of one band in the caller's arrays (the half sphere for a
 * real-mode plan); the stick, balance and group queries always describe the
 * whole sphere. */
/* Number of plane waves per band: the size of the cutoff sphere of Sec. 2,
 * eq. 3 (of its half H in the real mode). */
vloc_status vloc_plan_npw(vloc_plan plan, int64_t *npw);
/* hkl: npw*3 int32 (h, k, l) in canonical order: the sphere points of eq. 3,
 * the coefficient index of c and out. */
vloc_status vloc_plan_gvectors(vloc_plan plan, int32_t *hkl);
/* The columns that meet the sphere (the first pass of the compact 3-D FFT runs
 * only on them, Sec. 4.3; here z-sticks).
 * Stick table in canonical order: nsticks rows of (h, k, offset, count, lmin),
 * where the run [offset .. offset+count) of the whole sphere's canonical order
 * holds l = lmin .. lmin+count-1.  table may be NULL to query the count only. */
vloc_status vloc_plan_sticks(vloc_plan plan, int64_t *nsticks, int32_t *table);
/* Plane waves per stick group after the deal (the load-balance statistic of
 * the paper's Tab. 2, per workgroup instead of per process).  pw_per_group may
 * be NULL to query the count only. */
vloc_status vloc_plan_balance(vloc_plan plan, int64_t *ngroups, int64_t *pw_per_group);
/* Group of each stick (canonical stick order), nsticks int32: the column
 * distribution of Sec. 3.2 (greedy: sorted by plane-wave count, dealt in
 * turn), with stick groups in place of processes. */
vloc_status vloc_plan_stick_groups(vloc_plan plan, int32_t *group_of_stick);
/* Schedule of the plan's kernels (implementation choices, no paper quantity).
 * Sizes chosen by the plan: out[0..7] = {L1x, L2x, L1y, L2y, L1z, L2z,
 * sticks_per_group, band_chunk}; out[8..13] = {plane_rows, plane_threads,
 * plane_lds_bytes, nxo, plane_xwaves, plane_xmode} where nxo is the number of
 * occupied x-planes and plane_xmode is 1 (row buffers), 2 (lane quads), 3, 4 or 5
 * (whole plane) or 6 (parted plane; plane_rows is then the rows per part). */
vloc_status vloc_plan_layout(vloc_plan plan, int32_t out[14]);

/* ------------------------------------------------------- kernel timing */
/* When enabled, the plan records HIP events on its stream around each of its
 * kernel launches (stick forward K1, plane K2, stick backward K3).  Adds a few
 * microseconds per launch; meant for profiling runs. */
vloc_status vloc_plan_enable_timing(vloc_plan plan, int32_t enable);
/* Waits for the recorded events, writes the summed milliseconds of K1, K2, K3
 * into ms[3] and their launch counts into launches[3] (either may be NULL),
 * and resets the record. */
vloc_status vloc_plan_read_timing(vloc_plan plan, double ms[3], int64_t launches[3]);

/* ------------------------------------------------ energy and its gradients */
/* For the local-potential energy of weighted bands,
 *   E = sum_n w_n Re <c_n | V c_n>,  with out_n = V_loc c_n from vloc_apply,
 * the gradient with respect to V(j) is the weighted density
 *   dE/dV(j) = (1/N) sum_n w_n |psi_n(j)|^2   (psi_n as defined above),
 * and, V_loc being Hermitian, dE/d(Re c) + i dE/d(Im c) = 2 w_n (V c_n)(g)
 * (Sec. 2: the operator's action; its Hermiticity follows from V real).
 * Reductions accumulate in FP64 in a fixed order for either plan precision;
 * no atomics, so results are bitwise reproducible.  All pointers are device
 * pointers; the calls are stream-ordered like vloc_apply. */

/* e[n] = Re sum_g conj(a_n(g)) b_n(g), n < nbands.  a, b: [nbands][npw]
 * complex of the plan precision; e: double[nbands]. */
vloc_status vloc_band_dot(vloc_plan plan, const void *a, const void *b, int64_t nbands, double *e);
/* E[0] = sum_n w[n] x[n] over n < nbands (doubles). */
vloc_status vloc_weighted_sum(vloc_plan plan, const double *x, const double *w, int64_t nbands,
                              double *E);
/* rho(j) += s (1/N) sum_n w_n |psi_n(j)|^2 for n < nbands.  psi_n is recomputed
 * from c_n band chunk by band chunk inside the plane kernel and never stored;
 * partial sums are FP64.  rho: double [N3][N2][N1] (accumulated into);
 * w: double[nbands]; scale: one double s, or NULL for 1.  Needs the row-buffer
 * or whole-plane x pass (not plane_xmode 2); VLOC_E_INVALID otherwise. */
vloc_status vloc_density(vloc_plan plan, const void *c, int64_t nbands, const double *w,
                         const double *scale, double *rho);
/* The application and the weighted density of the same bands in one pass:
 * out[n] = V_loc c[n] as vloc_apply (bitwise the same result), and
 * rho(j) += (1/N) sum_n w_n |psi_n(j)|^2 as vloc_density, from the real-space
 * values the application computes anyway (Sec. 2: psi_n on the grid is the
 * intermediate of the operator), so the density costs no second transform.
 * rho: double [N3][N2][N1], accumulated into; w: double[nbands].  out and rho
 * must not overlap each other or the inputs (VLOC_E_ALIAS).  Needs the
 * row-buffer or whole-plane x pass (not plane_xmode 2); not for real-mode
 * plans. */
vloc_status vloc_apply_density(vloc_plan plan, const void *c, int64_t nbands, const void *V,
                               void *out, const double *w, double *rho);
/* y[i] = factor * s * x[i] for i < n (doubles, device); scale (one double s)
 * may be NULL for 1; y may equal x.  Used to apply the upstream gradient to a
 * density computed earlier. */
vloc_status vloc_scale_real(vloc_plan plan, const double *x, int64_t n, const double *scale,
                            double factor, double *y);
/* y_n = factor * s * w_n * x_n for n < nbands; w (double[nbands]) and scale
 * (one double s) may be NULL for 1; x, y: [nbands][npw] complex of the plan
 * precision; y may equal x. */
vloc_status vloc_scale_bands(vloc_plan plan, const void *x, int64_t nbands, const double *w,
                             const double *scale, double factor, void *y);

/* ------------------------------------------- diagnostic full-grid transforms */
/* The expansion of eq. 2 on the whole grid, through the compact transform of
 * Sec. 4.3: psi_r[n] = psi_n (same conventions as vloc_apply). */
vloc_status vloc_g2r(vloc_plan plan, const void *c, int64_t nbands, void *psi_r);
/* Its inverse on the sphere (the second transform of the operator, Sec. 2):
 * c_out[n](g) = (1/N) sum_j exp(+2 pi i g.j/N) psi_r[n](j) for g in S. */
vloc_status vloc_r2g(vloc_plan plan, const void *psi_r, int64_t nbands, void *c_out);

/* ------------------------------------------------------------- batches */
/* Several k-points of one crystal (same grid, cell, ecut and options, each
 * with its own cutoff sphere and band count) applied together (the paper's
 * balancing of uneven units, Sec. 3.2, carried to whole k-points; Sec. 1 on
 * aggregating the transforms of many bands).  A k-point with at least half a
 * band chunk of bands, or with enough bands that its z-planes fill the resident
 * plane workgroups eight times over, runs in launches of its own (its bands cut
 * into equal chunks); the bands of the smaller k-points are concatenated
 * (k-point order) and each chunk of them runs as ONE launch of each kernel,
 * whose workgroups take planes and stick groups of every k-point in it from one
 * work list.  All launches of a call are stream-ordered and can be replayed as
 * one HIP graph (vloc_batch_use_graph).  The members share one plane layout.
 * With the whole-plane layouts (plane_xmode 3 and 4) each member keeps its own
 * occupied x-planes (each launch segment carries them); with the others each
 * member covers the union of the k-points' occupied x-planes.  Either way a
 * member plan's own results (vloc_batch_plan) equal its part of the batch. */
typedef struct vloc_batch_s *vloc_batch; /* opaque; owned by the library */

/* nk in [1, 8]; kpts: nk*3 doubles (reduced coordinates, as for a plan).
 * opt (NULL = defaults) applies to every member; its band_chunk is the most
 * bands, counted over all k-points, of one launch (a call is cut into equal
 * chunks; 0 = automatic: the chunk's stick buffers within 256 MiB).  Errors as
 * for vloc_plan_create_ex; on error *batch is NULL. */
vloc_status vloc_batch_create(vloc_batch *batch, const int32_t grid[3], const double cell[9],
                              double ecut, int32_t nk, const double *kpts,
                              const vloc_options *opt);
/* Waits for the batch's stream, frees the batch and its member plans. */
vloc_status vloc_batch_destroy(vloc_batch batch);
/* Borrowed handle of member ik (queries, and stand-alone calls on its own
 * stream); valid until vloc_batch_destroy; vloc_plan_destroy refuses it. */
vloc_status vloc_batch_plan(vloc_batch batch, int32_t ik, vloc_plan *plan);
vloc_status vloc_batch_set_stream(vloc_batch batch, void *hip_stream);
/* out[i][n] = V_loc c[i][n] for every k-point i < nk and band n < nbands[i].
 * c, out: host arrays of nk device pointers ([nbands[i]][npw_i] complex of
 * the batch precision; entries of k-points without bands may be NULL);
 * nbands: host array of nk counts; V: device [N3][N2][N1] real.  No out may
 * overlap V, any c or another out (VLOC_E_ALIAS).  Stream-ordered and
 * asynchronous; calls on one batch must not run concurrently. */
vloc_status vloc_batch_apply(vloc_batch batch, const void *const *c, const int64_t *nbands,
                             const void *V, void *const *out);
/* With enable != 0, vloc_batch_apply records its launches once into a HIP
 * graph (captured on a private stream) and replays it on the batch's stream
 * while V, every c, out and band count stay the same; a change re-captures.
 * Kernel timing is not recorded on the graph path. */
vloc_status vloc_batch_use_graph(vloc_batch batch, int32_t enable);
/* Timing of the eager path, as vloc_plan_enable_timing / read_timing. */
vloc_status vloc_batch_enable_timing(vloc_batch batch, int32_t enable);
vloc_status vloc_batch_read_timing(vloc_batch batch, double ms[3], int64_t launches[3]);
/* out = {nk, band_chunk option, graphs captured, graph launches}. */
vloc_status vloc_batch_info(vloc_batch batch, int64_t out[4]);

/* Static description of a status code. */
const char *vloc_status_string(vloc_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char *vloc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VLOC_H */
