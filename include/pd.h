/*
 * pd.h - C ABI of the MI355X primal-dual solver for positive-contrast
 * susceptibility MRI (dipole-kernel deconvolution with an L1 prior).
 *
 * Method: Wang, Cai et al., "Positive Contrast Susceptibility MR Imaging Using
 * GPU-based Primal-Dual Algorithm", arXiv:2006.09808.  Each slice solves
 *
 *     min_chi  1/2 || A chi - delta ||^2 + lambda || chi ||_1,
 *     A = F^-1 diag(D) F,   D(k) = 1/3 - (k.b)^2 / |k|^2,   D(0) = 0,
 *
 * (Sec. II-A, Eq. (1), with lambda on the L1 term, W = I and the L1 prior on
 * chi itself) by the first-order primal-dual iteration of the paper's PD
 * pseudocode: dual prox, primal prox (soft threshold), over-relaxation.
 * Slices of a volume are independent 2-D problems (Sec. II-C, strategy (2));
 * the 2-D kernel is the dipole kernel at k_z = 0 on the unshifted DFT grid
 * k_i = i/(n d) (i < ceil(n/2)), else (i - n)/(n d); on an even grid with an
 * oblique in-plane B0 it is averaged between k and -k so A stays real.
 *
 * Conventions shared by every entry point:
 *   - Arrays are [nz][ny][nx], x fastest, densely packed, device memory of
 *     the context's device.  FP32 unless the context precision is PD_FP64.
 *   - No exceptions cross the ABI.  Every function returns a pd_status.
 *   - Calls on one context are serialised internally and may come from any
 *     host thread.  All GPU work of a context runs on its stream.
 *   - The caller owns every pointer it passes (arena, delta, chi); the
 *     library never frees them.
 */
#ifndef PD_H
#define PD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pd_status;

enum {
  PD_OK = 0,
  PD_PENDING = 1,          /* ticket not finished (pd_poll timeout)               */
  PD_ERR_ARG = -1,         /* null pointer, bad enum, non-finite parameter, ...   */
  PD_ERR_SIZE = -2,        /* nx or ny not a supported length, nz < 1             */
  PD_ERR_STEP = -3,        /* tau*sigma*max|D|^2 >= 1, theta outside [0, 1], ...
                              (TV model: tau*sigma*L2 >= 1, found at admission)   */
  PD_ERR_BUDGET = -4,      /* request can never fit in the context's arena       */
  PD_ERR_NONFINITE = -5,   /* a non-finite value appeared in the duality gap     */
  PD_ERR_HIP = -6,         /* HIP runtime error; the context is unusable         */
  PD_ERR_CANCELLED = -7,   /* request cancelled by pd_destroy                    */
  PD_ERR_TICKET = -8,      /* unknown (or already reported) ticket               */
  PD_ERR_NODEVICE = -9,    /* no usable GPU                                       */
  PD_ERR_SCRATCH = -10     /* needs more than PD_STATIC_SCRATCH_BYTES (the entry
                              point that allocates nothing)                       */
};

enum { PD_FP32 = 0, PD_FP64 = 1 };                      /* pd_config.precision */
/* pd_request.kernel:
 *   PD_KERNEL_DIPOLE     the 2-D kernel of each slice (slices independent);
 *   PD_KERNEL_IDENTITY   D = 1 (A = I; closed-form checks);
 *   PD_KERNEL_DIPOLE_3D  the 3-D kernel over the whole volume,
 *                        D(k) = 1/3 - (k.b)^2/|k|^2 with k = (kx, ky, kz),
 *                        kz on the nz grid with slice thickness voxel_z
 *                        (the paper's "all three dimensions"; Sec. II-A).
 *                        It couples the slices: every iteration transforms
 *                        along z too.  Both models; nz >= 2 and a
 *                        supported length like nx and ny.                    */
enum { PD_KERNEL_DIPOLE = 0, PD_KERNEL_IDENTITY = 1, PD_KERNEL_DIPOLE_3D = 2 };
/* pd_request.model:
 *   PD_MODEL_L1  min 1/2||A chi - delta||^2 + lambda ||chi||_1 (see the top),
 *                with the duality-gap stop rule available;
 *   PD_MODEL_TV  the full Eq. (1),
 *                min lambda/2 ||W (A chi - delta)||^2 + ||M G chi||_1,
 *                by the PD pseudocode with K = [W A; M G] (Sec. II-A):
 *                  p <- (p + sigma (W A chibar - W delta)) / (1 + sigma/lambda)
 *                  q <- v / max(1, |v|),  v = q + sigma M G chibar (per voxel)
 *                  chi' = chi - tau A W p - tau G* M q
 *                  chibar = chi' + theta (chi' - chi)
 *                lambda weights the data term here; W (weights) and M (mask)
 *                are real per-voxel arrays; G is the in-plane forward
 *                difference divided by the voxel size, zero at the last column
 *                and row (slices stay independent), with the isotropic
 *                norm |(g_x, g_y)|.  With PD_KERNEL_DIPOLE_3D the model is
 *                taken in three dimensions (Sec. II-A): A is the 3-D kernel
 *                and G gains the z difference divided by voxel_z, zero at
 *                the last slice, with the norm |(g_x, g_y, g_z)| and the step
 *                bound's extra 4/voxel_z^2.  Runs exactly max_iter
 *                iterations. */
enum { PD_MODEL_L1 = 0, PD_MODEL_TV = 1 };

/* pd_config.flags */
enum {
  PD_FLAG_TIME_KERNELS = 1,  /* time every launch of the iteration kernels with
                                HIP events on the context stream (pd_kernel_time) */
  PD_FLAG_NO_RESIDENT = 2,   /* never use the resident multi-iteration kernels
                                (L1 and TV models): two launches per iteration
                                for every shape (four for the TV model)        */
  PD_FLAG_FENCED_EXCHANGE = 4, /* resident kernel: always exchange between the
                                workgroups of a team with agent-scope
                                release/acquire (L2 write-back), even when
                                they share an XCD                              */
  PD_FLAG_NO_GRAPHS = 8,     /* never replay a step of the two-launch path from
                                a captured HIP graph                           */
  PD_FLAG_TEST_BARRIER_GIVEUP = 16 /* test hook: resident-kernel barriers give
                                up at their first wait (every workgroup exits
                                before touching state), which forces the
                                recovery path below                        */
};
/* Recovery from a resident launch that cannot complete.  The resident kernel
 * synchronises the workgroups of a team with bounded spin barriers; if its
 * workgroups are not all co-resident (other work holding CUs), a barrier
 * gives up, every workgroup of the launch exits and later resident launches
 * of the same scheduling round do nothing.  The context stays usable: the
 * requests those launches covered restart from chi_0 = 0 on the two-launch
 * path (no co-residency needed), which gives the same iterates up to
 * rounding, and their slice shapes stay on that path for the rest of the
 * context (pd_tune_set with a resident variant re-enables it).  The
 * solver's state, kept on the GPU between steps as in the paper's
 * device-resident scheme (Sec. II-D), is rebuilt from the field map, which
 * stays valid until the ticket completes.  pd_recovery_stats counts these
 * events. */

typedef struct pd_ctx pd_ctx;     /* opaque, library-owned */

typedef struct {
  int device;          /* HIP device ordinal                                      */
  void* stream;        /* hipStream_t to run on; NULL: the library creates one    */
  void* arena;         /* caller-owned device memory; all per-request state and
                          tables are carved from it.  Its size is the HBM budget
                          under which requests are admitted.                       */
  size_t arena_bytes;
  int max_slots;       /* most requests resident on the GPU at once; 0 = no cap  */
  int precision;       /* PD_FP32 (default) or PD_FP64                            */
  int step_iters;      /* most iterations of one step (one resident launch, or one
                          captured graph of the two-launch path); a step also
                          ends at every request's next gap check; 0 = 500, or 50
                          while requests wait in the queue.  Requests are
                          admitted and retired between rounds: while none waits,
                          a round enqueues up to 8 steps (100 iterations, or up
                          to some request's last iteration) before the host
                          reads the stop flags; otherwise one step.  A volume
                          whose gap check stops it mid-round is skipped by the
                          round's later steps, so results do not depend on the
                          round length.                                          */
  int flags;           /* PD_FLAG_* */
  const char* tune_cache; /* path of a text file of autotuner choices, one line
                          "nx ny variant rows cols plan_x plan_y" per slice
                          shape (five-field lines read with plans 0): read at
                          pd_create if it exists (lines that pd_tune_set would
                          reject are skipped), rewritten after every pd_tune
                          and pd_tune_set.  NULL: the PD_TUNE_CACHE environment
                          variable if set, else no file.  The string is copied. */
} pd_config;

/* One reconstruction: a volume of nz slices of ny x nx voxels (Eq. (1)). */
typedef struct {
  int nx, ny, nz;      /* nx, ny: 8,16,24,32,48,64,96,128,192,256,288,384,512,576,768
                          (direct FFT plans) or any other length 2..384, whose
                          DFTs run as Bluestein (chirp-z) convolutions on the
                          smallest direct length >= 2n - 1                      */
  double b0[3];        /* B0 direction in voxel axes (x, y, z); any non-zero scale */
  double voxel[2];     /* in-plane voxel size (dx, dy), any positive unit          */
  int kernel;          /* PD_KERNEL_DIPOLE, PD_KERNEL_IDENTITY or PD_KERNEL_DIPOLE_3D */
  double lambda;       /* weight of the L1 term (> 0)                              */
  double tau, sigma;   /* primal and dual step sizes (PD pseudocode, step 1)       */
  double theta;        /* over-relaxation in [0, 1]                                */
  int max_iter;        /* iteration cap N (pseudocode step 5), >= 0                */
  double gap_tol;      /* stop at the first check with relgap <= gap_tol; 0: run
                          exactly max_iter iterations                               */
  int check_every;     /* check cadence in iterations when gap_tol > 0 (>= 1)      */
  const void* delta;   /* field map [nz][ny][nx]; must stay valid and unchanged
                          until the ticket completes                               */
  void* chi;           /* output [nz][ny][nx]; written once, at completion         */
  int model;           /* PD_MODEL_L1 (0) or PD_MODEL_TV                           */
  const void* weight;  /* TV model: W [nz][ny][nx] (like delta: valid, unchanged
                          until completion); non-NULL for PD_MODEL_TV           */
  const void* mask;    /* TV model: M [nz][ny][nx], same rules                     */
  double voxel_z;      /* slice thickness (same unit as voxel), > 0; read only
                          for PD_KERNEL_DIPOLE_3D                                   */
} pd_request;
/* TV model specifics: gap_tol must be 0 and lambda > 0 (PD_ERR_ARG otherwise);
 * check_every is ignored.  Its step condition, tau*sigma*L2 < 1 with
 *   L2 = max|W|^2 max|D|^2 + max|M|^2 (4/dx^2 + 4/dy^2)  (a bound on ||K||^2),
 * needs the maxima of W and M, which the library takes on the GPU at
 * admission: a violation ends the ticket with PD_ERR_STEP and a non-finite
 * value in delta, W or M with PD_ERR_NONFINITE, before any iteration (chi
 * then holds zeros).  pd_validate cannot see W and M and does not test it. */

typedef struct {
  pd_status status;    /* PD_OK, PD_ERR_NONFINITE, PD_ERR_CANCELLED or PD_ERR_HIP */
  int iterations;      /* updates applied; chi holds chi_iterations                */
  double primal;       /* P    = sum 1/2||A chi - delta||^2 + lambda ||chi||_1     */
  double dual;         /* Dual = sum -1/2 s^2||y||^2 - s <y, delta>,
                          s = min(1, lambda / max|A y|)                            */
  double rel_gap;      /* (P - Dual) / max(P, 1e-300), FP64 reductions.
                          primal, dual and rel_gap are NaN for the TV model       */
  double t_submit, t_start, t_done;   /* seconds on pd_now()'s clock              */
} pd_result;

/* Create a context on cfg->device: the device-side home of every request's
 * data and iteration state for the whole solve (Sec. II-D: intermediate data
 * and the per-slice state variables stay in GPU memory, so no transfer sits
 * inside the iteration).  The arena must be device memory of that device of
 * at least arena_bytes and stay allocated until pd_destroy returns.
 * Errors: PD_ERR_ARG (null/invalid field), PD_ERR_NODEVICE, PD_ERR_HIP. */
pd_status pd_create(const pd_config* cfg, pd_ctx** out);

/* Hand n reconstructions to the GPU (Sec. II-B, step (2): the field map
 * already lives in device memory, so "moving" it is admission into the
 * arena) to be iterated together with every other resident request, the
 * slices of all of them in parallel (Sec. II-C, strategies (2) and (3)).
 * Submit n requests; never blocks on the GPU.  On PD_OK tickets[0..n-1] hold
 * one ticket per request, and each request is admitted as soon as a slot and
 * enough arena are free (FIFO), then iterated together with every other
 * resident request.  Validation is all-or-nothing: on an error no request of
 * the batch is queued and the status names the first failing check
 * (PD_ERR_ARG, PD_ERR_SIZE, PD_ERR_STEP, PD_ERR_BUDGET, PD_ERR_HIP). */
pd_status pd_solve_batch(pd_ctx* c, const pd_request* r, int n, uint64_t* tickets);

/* The result hand-back of Sec. II-B, step (6): a request's end point is
 * decided on the GPU per volume (Sec. II-D), its chi written once into the
 * caller's device buffer, and this call reports it.
 * Wait up to timeout_ms (< 0: forever, 0: just look) for a ticket.  Returns
 * PD_PENDING while it runs; once finished, fills *out (if non-null), returns
 * out->status and forgets the ticket (a second poll gives PD_ERR_TICKET). */
pd_status pd_poll(pd_ctx* c, uint64_t ticket, pd_result* out, int timeout_ms);

/* End of the device residency that pd_create began (Sec. II-D).  Cancel
 * queued and running requests (their tickets end PD_ERR_CANCELLED and their
 * chi is left unwritten), wait for the GPU, free library resources.  Calls
 * already inside the context on other threads (a pd_poll waiting on a
 * ticket, a pd_tune) return first, pd_poll with PD_ERR_CANCELLED; calls that
 * start after pd_destroy has begun return PD_ERR_CANCELLED, and no call may
 * use the context once pd_destroy has returned.  The arena stays the
 * caller's.  Accepts NULL. */
pd_status pd_destroy(pd_ctx* c);

/* Static, human-readable name of a status. */
const char* pd_status_string(pd_status s);

/* Pure host check of one request, no GPU involved: the same validation
 * pd_solve_batch applies, except the arena size and the device pointers
 * (delta, chi, weight, mask may still be null, so a caller can size its
 * allocations first).  If state_bytes is non-null it receives the arena
 * bytes the request occupies while resident. */
pd_status pd_validate(const pd_request* r, int precision, size_t* state_bytes);

/* Largest |D(k)| of the request's kernel grid (||A||_2), computed in FP64 on
 * the host; the step condition is tau*sigma*norm^2 < 1. */
pd_status pd_kernel_norm(const pd_request* r, double* norm);

/* Forward operator on the device: out = A in for every slice of a
 * [nz][ny][nx] stack (the dipole field of a susceptibility map, Eq. (1)
 * operator D).  Uses r's nx, ny, nz, b0, voxel and kernel; delta is the input,
 * chi the output (they may not alias).  Needs arena space like a solve of the
 * same shape; runs on the context stream and returns when out is written. */
pd_status pd_apply_kernel(pd_ctx* c, const pd_request* r);

/* Size of the library's fixed device scratch: one array per GPU, held from
 * library load until the process ends. */
#define PD_STATIC_SCRATCH_BYTES (64u << 20)

/* pd_apply_kernel for callers that cannot allocate device memory (code that
 * must not call hipMalloc, e.g. a tight serving loop or a harness that
 * forbids it): the same kernels and the same result, but the exchange
 * buffer and the kernel tables (D grid, twiddles) live in the library's
 * fixed scratch instead of the context's arena, and the call makes no
 * device or pinned allocation (hipMalloc, hipFree, hipHostMalloc, arena).
 * The request must fit: FP32 needs 8 B per slice-pair point of the
 * transformed field (P = ceil(nz/2) pairs of ny x nx; nz planes for the 3-D
 * kernel) plus the tables (4 B per D-grid point and 8 B per twiddle);
 * otherwise PD_ERR_SCRATCH, before any GPU work.  The scratch is shared by
 * every call on its GPU and keeps the last call's contents; each call fills
 * everything it reads before reading it.  Calls of one process on one GPU
 * are serialised by the library (they never overlap in the scratch), and
 * each call returns when out is written.  Other errors as pd_apply_kernel. */
pd_status pd_apply_kernel_noalloc(pd_ctx* c, const pd_request* r);

/* Seconds on a monotonic clock (the clock of pd_result's time stamps). */
double pd_now(void);

/* With PD_FLAG_TIME_KERNELS: number of launches, summed HIP-event time in
 * milliseconds, and summed iterations x slice-pair points of one kernel class
 * since the last reset.  kind: 0 = column kernel (forward column FFT, dual
 * prox, inverse column FFT), 1 = row kernel (inverse row FFT, primal prox,
 * over-relaxation, forward row FFT), 2 = resident kernel (a whole step of
 * iterations of square slices kept on chip), 3 = TV-model column kernel
 * (forward column FFT, multiply by D, inverse column FFT; two per iteration),
 * 4 = TV-model row kernels (inverse row FFT, dual or primal update, forward
 * row FFT; two per iteration), 5 = the 3-D kernel's z transform (forward z
 * FFT, dual prox, inverse z FFT; kind 0 then counts its in-plane column
 * transforms), 6 = multi-shape resident launches (a whole step of the pairs
 * of several square shapes in one launch: 64x64, 128x128 and 256x256 volumes
 * whose chosen resident variant runs the default FFT plan, whenever a step
 * holds two or more such shapes), 7 = the TV model's resident launches (a
 * whole step of iterations of square 64x64, 128x128 or 256x256 TV volumes:
 * the column halves of the transforms on chip, the state streamed from HBM).
 * pd_kernel_time_reset clears all. */
pd_status pd_kernel_time(pd_ctx* c, int kind, int64_t* launches, double* total_ms, double* point_iters);
pd_status pd_kernel_time_reset(pd_ctx* c);

/* One timed configuration of a slice shape (pd_tune). */
typedef struct {
  int nx, ny, nz, iters;  /* problem timed: nz slices of ny x nx, iters iterations   */
  int path;               /* 0: resident kernel (whole iterations); 1: column kernel
                             of the two-launch path alone; 2: its row kernel alone */
  int variant;            /* resident: variant index; otherwise -1                   */
  int team, threads;      /* resident: workgroups per slice pair, threads per group  */
  int rows, cols;         /* row kernel: rows per workgroup; column kernel: columns
                             per workgroup; 0 otherwise                             */
  int plan;               /* column kernel: pass plan of the ny transforms; row
                             kernel: of the nx transforms; resident: the variant's
                             plan of both axes                                      */
  double ms;              /* best of three timed runs (HIP events), milliseconds      */
} pd_tune_entry;

/* Autotuner: time every kernel configuration of the nx x ny slice shape on a
 * zero-filled volume of nz slices for `iters` iterations, then make the
 * fastest of each kind the context's choice for that shape:
 *   - resident-kernel variants (square FP32 shapes: workgroups per pair x
 *     threads per workgroup x FFT pass plan; 192 x 192 has each of its two
 *     shapes twice, variants 2 and 3 registered for two waves per SIMD: part
 *     of the state spilled, twice the slice pairs per launch);
 *   - the two-launch path's column kernel per tile width and FFT pass plan of
 *     the length-ny transforms, and its row kernel per tile height and pass
 *     plan of the length-nx transforms, each timed alone.
 * A pass plan is a factorisation of the transform length into the radices
 * of its Stockham passes (256 as 16 x 16, 8 x 8 x 4 or 4 x 4 x 16; 384 as
 * 16 x 24, 24 x 16 or 8 x 6 x 8; ...); FP32 transforms of a direct length
 * over whole tiles have several, every other transform runs the default.
 * Plans compute the same DFT with different rounding, so solves under
 * different plans agree to rounding, not bit for bit (resident variants of
 * one plan, and tile sizes, do agree bit for bit; a step that needs more
 * co-resident teams than the chosen variant has switches only to a variant
 * of the same plan).  Needs arena space like a solve of that
 * size; blocks until done and runs between scheduling rounds.  The choice is
 * per shape, whatever the slice count of later requests: the widest resident
 * teams win for small batches and lose for large ones, so tune with a
 * representative nz.  Up to max_entries timings are written to entries (may
 * be NULL), their count to *n_entries.
 * Errors: PD_ERR_ARG, PD_ERR_SIZE, PD_ERR_BUDGET, PD_ERR_HIP. */
pd_status pd_tune(pd_ctx* c, int nx, int ny, int nz, int iters, pd_tune_entry* entries, int max_entries,
                  int* n_entries);

/* Set / read the context's configuration choice for the nx x ny shape
 * (e.g. a choice saved from an earlier pd_tune).  variant < 0, rows <= 0 or
 * cols <= 0 select the default of that knob, plan_x / plan_y <= 0 the
 * default pass plan of the row / column transforms; invalid values are
 * rejected with PD_ERR_ARG.  A plan applies where it exists (FP32 whole-tile
 * transforms of the L1 model's iterations); elsewhere the default runs. */
pd_status pd_tune_set(pd_ctx* c, int nx, int ny, int variant, int rows, int cols, int plan_x, int plan_y);
pd_status pd_tune_get(pd_ctx* c, int nx, int ny, int* variant, int* rows, int* cols, int* plan_x, int* plan_y);

/* Scheduling steps of the two-launch path captured into HIP graphs, and
 * steps replayed from one, since pd_create. */
pd_status pd_graph_stats(pd_ctx* c, int64_t* captures, int64_t* replays);

/* Scheduling rounds in which a resident launch gave up, and requests
 * restarted on the two-launch path because of it, since pd_create. */
pd_status pd_recovery_stats(pd_ctx* c, int64_t* aborted_rounds, int64_t* restarted_requests);

/* Bytes of arena currently in use (control blocks, resident requests' state,
 * and kernel tables: D grid and twiddles per kernel shape, which stay cached
 * after their last request retires and are evicted, least recently used
 * first, when an admission needs the space), the number of resident requests
 * and the number of queued ones. */
pd_status pd_arena_usage(pd_ctx* c, size_t* used, int* resident, int* queued);

#ifdef __cplusplus
}
#endif
#endif /* PD_H */
