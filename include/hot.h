/*
 * libhot -- one classical RK4 time step of the Fourier-Galerkin
 * Navier-Stokes right-hand side on a triply periodic N^3 grid, on one
 * MI355X (gfx950).
 *
 * The method (Mortensen, arXiv 1607.00850):
 *   du_k/dt = (u x w)^_k - nu |k|^2 u_k - k (k . (u x w)^_k) / |k|^2
 * (Eq. NSfinal, pressure eliminated by Eq. pressure, w = curl u), evaluated
 * pseudo-spectrally with the transform pair of Eq. ffteq on the mesh of
 * Eq. realmesh and the wavenumbers of Eq. wavemesh, dealiased with the 2/3
 * rule, and advanced with classical fourth-order Runge-Kutta (Sec. 2).
 *
 * Layouts (all device memory, row-major, contiguous):
 *   spectral  uhat[3][N][N][N/2+1]  complex (interleaved re, im), index
 *             [c][kx][ky][kz]; kx, ky in FFT order (index j <-> k = j for
 *             j <= N/2, j - N above), kz = 0..N/2.  This is the spectral
 *             array of the slab transform (Sec. 3.3) on a single rank.
 *   physical  u[3][N][N][N] real, index [c][x][y][z] at x_i = 2 pi i / N.
 *   element type: double (HOT_F64) or float (HOT_F32).
 *
 * Ownership: the caller allocates inputs, outputs and the workspace (e.g.
 * torch tensors); the library never allocates or frees device memory, and
 * hot_run only enqueues kernels on the given stream (two documented
 * exceptions wait for it: CHECK_FINITE plans, and an IMPLICIT call's looks at
 * its stopping flags, see HOT_OP_IMPLICIT).  All device pointers must be
 * 256-byte aligned.
 *
 * Thread safety: a plan may be used from one host thread at a time.  Two
 * hot_run calls that share a workspace must be ordered on one stream.
 */
#ifndef HOT_H
#define HOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOT_ABI_VERSION 3

/* Return codes. */
#define HOT_OK 0
#define HOT_E_INVALID (-1)     /* bad argument (null, odd N, nu < 0, dt <= 0, bad enum, ...) */
#define HOT_E_UNSUPPORTED (-2) /* valid request the library does not implement (e.g. an N) */
#define HOT_E_WORKSPACE (-3)   /* workspace pointer null or misaligned */
#define HOT_E_HIP (-4)         /* a HIP call failed; hot_last_hip_error() has the code */
#define HOT_E_NONFINITE (-5)   /* HOT_FLAG_CHECK_FINITE: a result holds a NaN or an infinity */
#define HOT_E_TOOBIG (-7)      /* hot_run_noalloc: the plan's workspace exceeds the static scratch */
#define HOT_E_NOCONVERGE (-6)  /* IMPLICIT: an instance hit max_iter sweeps (its last iterate is kept);
                                  reported by hot_implicit_stats, and by hot_run for CHECK_FINITE plans */

/* Element type. */
#define HOT_F64 0
#define HOT_F32 1

/* Dealiasing (Sec. 4 names the technique only as Tarang's; read as the
 * 2/3 rule): TWO_THIRDS keeps mode k iff 3|k_i| < N on every axis.
 * NONE keeps every mode except the Nyquist planes (|k_i| = N/2). */
#define HOT_DEALIAS_TWO_THIRDS 0
#define HOT_DEALIAS_NONE 1

/* Operations.
 *  R2C  physical u -> spectral uhat_k = sum_x u(x) e^{-i k.x}
 *       (Eq. ffteq, forward, unnormalised; every mode kept, no dealiasing).
 *  C2R  spectral -> physical u(x) = N^-3 sum_k uhat_k e^{i k.x} (Eq. ffteq,
 *       inverse; the imaginary parts of the kz = 0 and N/2 coefficients
 *       are ignored, as for any real inverse transform).
 *  RHS  spectral uhat -> spectral du/dt of Eq. NSfinal.  The input is first
 *       projected onto the retained modes (the Galerkin space of the
 *       dealiased method); the output is zero outside them.
 *  RK4  spectral uhat -> spectral uhat after nsteps classical RK4 steps of
 *       size dt (Sec. 2), input projected as for RHS.  in == out allowed.
 *  IMPLICIT  spectral uhat -> spectral uhat after nsteps implicit-midpoint
 *       steps (Crank-Nicolson on the viscous term), an implicit alternative
 *       to the RK4 integration of Sec. 2: with m = (u^n + u^{n+1})/2,
 *       u^{n+1} - u^n = dt F(m), F the right-hand side of Eq. NSfinal.  Each
 *       step is solved by Picard sweeps on the increment d = u^{n+1} - u^n,
 *         d <- [dt F_NL(u^n + d/2) - 2a u^n] / (1 + a),  a = dt nu |k|^2 / 2,
 *       F_NL the projected, dealiased nonlinear term, until
 *       ||d_new - d|| <= tol ||d_new|| (L2 norms of the real field) or
 *       max_iter sweeps.  The first sweep starts from the polynomial
 *       through the last m = min(4, steps so far) increments, one step
 *       ahead: 0, d^{n-1}, 2 d^{n-1} - d^{n-2},
 *       3 d^{n-1} - 3 d^{n-2} + d^{n-3}, then
 *       4 d^{n-1} - 6 d^{n-2} + 4 d^{n-3} - d^{n-4} (or, from the third
 *       step, the surrogate's warm start, see hot_set_surrogate; with
 *       HOT_FLAG_KEEP_HISTORY the history carries over from the previous
 *       call).  Each instance stops on
 *       its own: the kernels of a sweep return at once for an instance that
 *       has stopped.  Sweeps are enqueued in rounds of K (hot_set_variant
 *       pass "imp_decide", default 2); after each round but the last an
 *       eager call copies the stopping flags to the host, waits for them,
 *       and enqueues no further sweeps for a size whose instances have all
 *       stopped (a sweep launches every block even when they all return at
 *       once).  K = 0, and every call captured by hot_graph_create, enqueue
 *       all max_iter sweeps and never wait.  The sweep counts stay on the
 *       device (hot_stats, hot_implicit_stats).  in == out allowed. */
#define HOT_OP_R2C 0
#define HOT_OP_C2R 1
#define HOT_OP_RHS 2
#define HOT_OP_RK4 3
#define HOT_OP_IMPLICIT 4

/* Flags (hot_desc.flags).
 * KEEP_HISTORY (IMPLICIT only): the increments of earlier steps stay in the
 * workspace between calls, so a call continues the predictor history of the
 * previous call on the same plan and workspace; the caller passes the state
 * that call returned.  Without it every call starts without history. */
#define HOT_FLAG_KEEP_HISTORY 1
/* CHECK_FINITE (RHS, RK4, IMPLICIT): hot_run ends by scanning every
 * instance's result (its retained modes) for NaN and infinity and returns
 * HOT_E_NONFINITE if it finds one; this costs one synchronisation, so such a
 * plan cannot be captured in a graph.  The workspace grows by 256 bytes. */
#define HOT_FLAG_CHECK_FINITE 2

typedef struct hot_desc {
  int32_t abi_version; /* HOT_ABI_VERSION */
  int32_t batch;       /* number of instances, >= 1 */
  const int32_t* n;    /* host array [batch]: points per axis of each instance */
  double nu;           /* kinematic viscosity (>= 0); Sec. 4 uses Re = 1600 -> nu = 1/1600 */
  double dt;           /* time step (> 0, RK4 and IMPLICIT); Sec. 4 uses 0.001 */
  int32_t dtype;       /* HOT_F64 or HOT_F32 */
  int32_t dealias;     /* HOT_DEALIAS_* (RHS and RK4) */
  int32_t op;          /* HOT_OP_* */
  int32_t flags;       /* HOT_FLAG_* (KEEP_HISTORY: IMPLICIT only; CHECK_FINITE: RHS, RK4, IMPLICIT) */
  double tol;          /* IMPLICIT: relative stopping tolerance (> 0); ignored otherwise */
  int32_t max_iter;    /* IMPLICIT: sweeps per step at most (>= 1); ignored otherwise */
  int32_t reserved;    /* must be 0 */
} hot_desc;

typedef struct hot_plan_s* hot_plan_t;

/* Per-instance statistics of a hot_run call (RHS, RK4, IMPLICIT), written
 * on the stream into a caller's device array [batch] (stats_dev):
 *   energy       E = (1/2N^6) sum_k |u_k|^2, the kinetic energy by Parseval
 *                under Eq. ffteq, of the state (the RHS input, the RK4 and
 *                IMPLICIT result; sums over the full spectrum, FP64);
 *   dissipation  eps = nu (1/N^6) sum_k |k|^2 |u_k|^2 = nu <|w|^2> of it,
 *                the rate at which the viscous term of Eq. NSfinal removes
 *                energy;
 *   sweeps       IMPLICIT: Picard sweeps summed over the call's steps;
 *   nonconv      IMPLICIT: steps that stopped at max_iter (0 for the others). */
typedef struct hot_stats {
  double energy;
  double dissipation;
  int32_t sweeps;
  int32_t nonconv;
} hot_stats;

/* Supported sizes: N in {8, 16, 18, 24, 32, 36, 48, 54, 64, 128, 256, 512, 1024}. */

/* Validate d, build a plan and report the workspace size in bytes.
 * The plan copies d->n.  On error *out is set to NULL.
 * Errors: HOT_E_INVALID, HOT_E_UNSUPPORTED. */
int hot_plan(const hot_desc* d, hot_plan_t* out, size_t* workspace_bytes);

/* Enqueue the planned operation on stream (a hipStream_t; NULL = default).
 * The call never synchronises, except for a CHECK_FINITE plan and the looks
 * at the stopping flags of an IMPLICIT call (HOT_OP_IMPLICIT).
 * in[i], out[i]: device pointers of instance i (layouts above; R2C reads
 * physical and writes spectral, C2R the reverse, RHS/RK4/IMPLICIT spectral
 * both).  Instances must not overlap each other (in[i] == out[i] is allowed).
 * workspace: device buffer of at least the planned size.  nsteps: RK4 or
 * IMPLICIT steps (>= 0; ignored by other ops).  stats_dev: NULL, or a
 * device array of batch hot_stats records (8-byte aligned; RHS, RK4 and
 * IMPLICIT only) filled on the stream at the end of the call.  Inputs must
 * stay valid until the stream reaches the end of the call.
 * Batches: for RHS, RK4 and IMPLICIT, instances of equal N run together, each pass as
 * one launch over all of them (the instance is a grid dimension).  The
 * device tables of their in/out pointers live in the workspace; every call
 * writes them on the stream with a small kernel whose arguments carry the
 * pointers (no host synchronisation).
 * Errors: HOT_E_INVALID (null plan/pointer, nsteps < 0, stats_dev for
 * R2C/C2R or misaligned), HOT_E_WORKSPACE, HOT_E_HIP (launch failure; the
 * plan keeps the HIP error code).  A CHECK_FINITE plan, which synchronises,
 * also returns HOT_E_NONFINITE (the whole call ran and a result holds a NaN
 * or an infinity) or, for IMPLICIT, HOT_E_NOCONVERGE (some step of some
 * instance stopped at max_iter), the first taking precedence. */
int hot_run(hot_plan_t p, void* const* in, void* const* out, void* workspace, int32_t nsteps, void* stats_dev,
            void* stream);

/* hot_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation with the library's own static scratch, 16 MiB per device
 * (held from the first use on a device until the process ends), as the
 * workspace.  It calls no allocating routine.  Every call on a device shares
 * that device's scratch, which keeps the last call's contents: calls that
 * overlap on one device race (order them on one stream), and a plan with
 * HOT_FLAG_KEEP_HISTORY is rejected (HOT_E_UNSUPPORTED).  Plans whose
 * workspace (hot_plan's workspace_bytes) exceeds 16 MiB return HOT_E_TOOBIG;
 * single instances up to N = 64 fit in FP32 and up to N = 48 in FP64 for
 * RK4.  Per-pass profiling is not recorded.  Otherwise as hot_run. */
int hot_run_noalloc(hot_plan_t p, void* const* in, void* const* out, int32_t nsteps, void* stats_dev, void* stream);

/* A captured hot_run: the whole operation (every pass of every instance and
 * step) recorded once into a HIP graph and replayed with one launch.
 * hot_graph_create captures on stream, which must not be the legacy default
 * stream (NULL).  With several distinct N each size is a branch of the graph
 * (see the "graph" variant of hot_set_variant); the plan creates one side
 * stream per size for the capture (default priority) and keeps them until
 * hot_destroy.  stats_dev: NULL or as for hot_run.  The graph keeps the
 * pointers it was created with: a replay rewrites the pointer tables itself,
 * so hot_run calls with other arrays on the same workspace between replays
 * do not change what a replay reads and writes.  Per-pass profiling is
 * not recorded inside graphs.  Errors as hot_run; HOT_E_UNSUPPORTED for
 * plans with HOT_FLAG_CHECK_FINITE (it needs the host) or
 * HOT_FLAG_KEEP_HISTORY (a replay would not continue the history). */
typedef struct hot_graph_s* hot_graph_t;
int hot_graph_create(hot_plan_t p, void* const* in, void* const* out, void* workspace, int32_t nsteps,
                     void* stats_dev, void* stream, hot_graph_t* graph);
int hot_graph_launch(hot_graph_t graph, void* stream);
int hot_graph_destroy(hot_graph_t graph);

/* Autotuner: for every distinct N of the plan and every column-tiled pass
 * (x inverse with the curl, y inverse, y forward, x forward), time each
 * column-width variant reps times
 * on the workspace (which must be the planned size; the caller's arrays are
 * not touched) and keep the fastest for later hot_run calls.  For RK4 and
 * RHS it also times the x forward pass fused with the stage update (pass
 * "x_fwd_rk": the nonlinear term stays in registers) against the two
 * separate passes and keeps the faster, and for the sizes that have it the
 * fused y-z pass against the separate y and z passes (a plan with several
 * distinct N keeps the fused pass untimed: its sizes run side by side and
 * share the HBM, which the fused pass spares).  Synchronises the stream.
 * hot_tuned_width reports the chosen columns per block of a pass for
 * instance i (for x_fwd_rk: 0 when the separate passes were kept), or a
 * negative error code. */
int hot_tune(hot_plan_t p, void* workspace, void* stream, int32_t reps);
int hot_tuned_width(hot_plan_t p, int32_t instance, int32_t pass);

/* Set what hot_tune would choose, for every size of the plan: for a
 * column-tiled pass the width variant 0 (narrow), 1 (default) or 2 (wide),
 * and 3..5 the same widths with one output per block for the y forward pass
 * on packed rows (c0, c1, c2 separated by three blocks) and for the x inverse
 * with the curl at N > 64 (six blocks per tile instead of three);
 * for x_fwd_rk -1 (separate x_fwd and rk_stage passes), 0, 1 or 2 (fused,
 * at half, the default or a quarter of the default width); for z_cross 1
 * (the default: the y and z passes carry u and w as packed pairs of complex
 * lines), 2 (packed pairs into the z pass, which stores c0, c1, c2 as three
 * component rows for the y forward pass), 3 (six component rows through the
 * y passes; the z pass packs them into complex lines on load and stores
 * c0, c1, c2 as component rows) or 0 (six component rows, the z pass
 * completing the Hermitian halves in LDS), hot_tune timing the four over
 * the y inverse, z and y forward passes; for "graph" (no kernel of its own)
 * the batch schedule: 1 (the default) graphs hot_graph_create captures from
 * then on have one branch per distinct N, forked from and joined back into
 * the capturing stream, so the passes of small sizes run beside those of
 * large ones; 0 the sizes one after another; 2 (RK4 plans in FP32 with the
 * 2/3 rule and at most 8 distinct N, each of 16, 18, 24, 32, 36, 48, 54 or
 * 64) every pass of every instance and step of a hot_run or captured call
 * in one launch of a persistent kernel (pass "persistent": a queue of work
 * items in the workspace, each pass as in the fused schedule, Sec. 2's RK4
 * on Eq. NSfinal), eager or captured; for "persistent" (the plans of
 * schedule 2) the bound of the kernel's waits in polls, 0 (the default) for
 * about a second: a wait past it raises an error flag, no wait follows and
 * the call's outputs from then on are NaN (a small bound forces that path for
 * tests); for "imp_decide" (IMPLICIT plans only) the sweeps per round
 * between an eager call's looks at the stopping flags, K >= 0 (default 2; 0:
 * never look, enqueue max_iter sweeps).  hot_tuned_width reports these
 * settings for the non-tiled passes.  Host only.  Errors: HOT_E_INVALID. */
int hot_set_variant(hot_plan_t p, int32_t pass, int32_t variant);

/* IMPLICIT statistics of the plan's last hot_run (or graph capture), per
 * instance i (host arrays of p's batch size, either may be NULL): sweeps[i] =
 * Picard sweeps summed over the call's steps, nonconv[i] = steps that stopped
 * at max_iter.  Waits for the stream of that call, then copies the counters
 * from its workspace (a graph replay must have finished before this call).
 * Returns HOT_OK, or HOT_E_NOCONVERGE when some nonconv[i] > 0.
 * Errors: HOT_E_INVALID (null plan, op not IMPLICIT), HOT_E_HIP. */
int hot_implicit_stats(hot_plan_t p, int32_t* sweeps, int32_t* nonconv);

/* ------------------------------------------------------------------------
 * Per-mode MLP surrogate for the implicit step (not in the paper: Sec. 2
 * leaves the integrator open, and a Picard iteration needs a starting
 * guess).  Once two earlier increments D1 (newest) and D2 exist, the first
 * sweep of a step starts from
 *     d = 2 D1 - D2 + s MLP(f),   s = ||D1_k|| over the 3 complex components,
 * instead of the plain predictor (2 D1 - D2, or the extrapolation of three
 * or four increments once they exist: the network corrects the linear
 * extrapolation it was trained on, whatever the history depth).  MLP: 32 ->
 * 256 -> 256 ->
 * 256 -> 6, tanh hidden layers, BF16 MFMA operands with FP32 accumulation.
 * Features f of mode k, a = dt nu |k|^2 / 2 (all 0 when s = 0):
 *   f[0:6] D1/s, f[6:12] D2/s, f[12:18] ((1 - a) D1 + 2 a u)/s,
 *   f[18:24] u/||u_k||, f[24] s/||u_k||, f[25:28] k/N, f[28] a, f[29:32] 0
 * (re, im of components x, y, z; u the state at the start of the step).
 * The output y holds the correction in the same (re, im) x 3 order.
 *
 * Parameters: one device FP32 vector of hot_mlp_param_count() values,
 *   W1[256][32] b1[256] W2[256][256] b2[256] W3[256][256] b3[256]
 *   W4[6][256] b4[6]    (weights W[out][in], row-major).
 * All pointers are device pointers, 16-byte aligned (workspaces 256). */

/* Number of FP32 parameters, and bytes of the packed inference copy. */
int32_t hot_mlp_param_count(void);
size_t hot_mlp_packed_bytes(void);

/* params -> packed (BF16 weights, FP32 biases), enqueued on stream. */
int hot_mlp_pack(const float* params, void* packed, void* stream);

/* y[rows][6] = MLP(x[rows][32]) with the packed parameters (the fused
 * inference kernel the implicit step uses).  Errors: HOT_E_INVALID. */
int hot_mlp_forward(const void* packed, const float* x, float* y, int64_t rows, void* stream);

/* Training.  hot_mlp_grad: mean squared error of MLP(x) against t[rows][6]
 * into *loss (device float) and its gradient with respect to params into
 * grad (hot_mlp_param_count floats), by backpropagation with BF16 MFMA
 * products; ws: device workspace of hot_mlp_train_bytes(rows) bytes.
 * hot_mlp_adam: one bias-corrected Adam update (step >= 1) of params with
 * moment buffers m, v (param_count floats each, zero before step 1). */
size_t hot_mlp_train_bytes(int32_t rows);
int hot_mlp_grad(const float* params, const float* x, const float* t, int32_t rows, float* grad, float* loss,
                 void* ws, void* stream);
int hot_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                 float beta2, float eps, void* stream);

/* Training data of one N^3 field (2/3 rule): the features of every retained
 * mode, rows = hot_mlp_dataset_rows(N) of them in canonical (kx, ky, kz)
 * order, into x[rows][32]; when d is not NULL the targets
 * (d - (2 d1 - d2)) / s into t[rows][6] (0 where s = 0); when s is not NULL
 * the scales s = ||d1_k|| into s[rows].  u: the state at
 * the start of a step; d1, d2: the increments of the two steps before it
 * (newest first); d: the step's own increment.  Canonical spectral layout,
 * element type dtype; x, t FP32.  Errors: HOT_E_INVALID. */
int64_t hot_mlp_dataset_rows(int32_t N);
int hot_mlp_dataset(int32_t N, int32_t dtype, const void* u, const void* d1, const void* d2, const void* d, double nu,
                    double dt, float* x, float* t, float* s, void* stream);

/* Use the packed surrogate (hot_mlp_pack output, device memory the caller
 * keeps alive) for the warm start of an IMPLICIT plan's later hot_run calls;
 * NULL returns to the plain predictor.  Host only.
 * Errors: HOT_E_INVALID (null plan, op not IMPLICIT, misaligned pointer). */
int hot_set_surrogate(hot_plan_t p, const void* packed);

/* Diagnostics of every instance's spectral field in[i] (canonical layout, the
 * plan's element type and N): out[2i] = E = (1/2N^6) sum_k |u_k|^2, the
 * kinetic energy by Parseval under Eq. ffteq, and out[2i+1] = eps =
 * nu (1/N^6) sum_k |k|^2 |u_k|^2 = nu <|omega|^2>, the rate at which the
 * viscous term of Eq. NSfinal removes energy (sums over the full spectrum,
 * written over the half spectrum).  out: device doubles [batch][2],
 * written on stream (FP64 sums in a fixed order).  The first 2 KiB of the
 * workspace serve as scratch (one instance after the other): between
 * hot_run calls nothing lives there, kept implicit histories included.
 * Errors: HOT_E_INVALID, HOT_E_WORKSPACE, HOT_E_HIP. */
int hot_diagnostics(hot_plan_t p, void* const* in, void* workspace, double* out, void* stream);

/* ------------------------------------------------------------------------
 * One share of a slab-decomposed field (Sec. 3, "Mesh decomposition" and
 * "Three dimensional Fourier transforms with MPI").  nranks shares split one
 * N^3 field: in physical space share r holds the x planes
 * [r*nx, (r+1)*nx), nx = N/nranks; in wavenumber space it holds a slab of
 * kz, the second of the two alignments the paper names for the last
 * transform (the paper's own code distributes ky).  So the x and y transforms
 * are local and one all-to-all per direction sits next to the z transform:
 * six components go from the wavenumber slabs to the physical slabs after
 * the inverse y pass, three come back after the forward z pass.  The library
 * runs the local passes; the caller moves the blocks between the shares
 * (RCCL all-to-all, one per component; or device copies when the shares
 * share a device).  The retained kz [0, Mz) are split in chunks of
 * ceil(Mz/nranks); share r holds kz0 = r*chunk onwards.
 * ------------------------------------------------------------------------ */

/* Where the exchanged blocks sit (byte offsets into the share's workspace).
 * Both buffers are [6 components][nranks blocks][nx][N][pitch] elements;
 * block q of a component is block_bytes long, components are comp_bytes
 * apart.  Forward exchange (after HOT_SLAB_INVERSE), for c = 0..5: send
 * block q of component c of the send buffer to share q, into block `rank` of
 * component c of its receive buffer.  Backward exchange (after
 * HOT_SLAB_CROSS), for c = 0..2: send block q of component c of the receive
 * buffer to share q, into block `rank` of component c of its send buffer. */
typedef struct hot_slab_layout {
  int32_t nranks, rank;
  int32_t nx;     /* x planes of each physical slab: N / nranks */
  int32_t kz0;    /* first kz of this share */
  int32_t nkz;    /* kz extent of the share's canonical in/out arrays: chunk,
                     or for the last share N/2+1 - kz0 (the truncated kz too) */
  int32_t mz;     /* retained kz of this share: kz0 .. kz0 + mz - 1 */
  int32_t chunk;  /* retained kz per share (the last share may hold fewer) */
  int32_t pitch;  /* z pitch of the exchanged blocks (>= chunk) */
  size_t send_offset, recv_offset, comp_bytes, block_bytes;
} hot_slab_layout;

/* Plan share `rank` of `nranks` of one field.  d as for hot_plan with
 * batch = 1, op HOT_OP_RHS or HOT_OP_RK4, flags = 0.  N must be a multiple
 * of nranks and every share must hold at least one retained kz
 * ((nranks - 1) * chunk < Mz), else HOT_E_UNSUPPORTED.  The workspace holds
 * the share's compact state and both exchange buffers.  hot_run,
 * hot_graph_create and hot_diagnostics return HOT_E_UNSUPPORTED on a plan
 * with nranks > 1; hot_tune (it times the local passes only, on the
 * workspace: tune before HOT_SLAB_GATHER), hot_set_variant, profiling and
 * hot_pass_bytes work.  Host only. */
int hot_plan_slab(const hot_desc* d, int32_t nranks, int32_t rank, hot_plan_t* out, size_t* workspace_bytes);
int hot_slab_layout_of(hot_plan_t p, hot_slab_layout* out);

#define HOT_SLAB_GATHER 0  /* in (canonical share [3][N][N][nkz]) -> state   */
#define HOT_SLAB_INVERSE 1 /* x and y inverse passes -> send buffer           */
#define HOT_SLAB_CROSS 2   /* z passes and u x omega, in the receive buffer   */
#define HOT_SLAB_FORWARD 3 /* y and x forward passes, the stage update        */
#define HOT_SLAB_SCATTER 4 /* state (RK4) or right-hand side (RHS) -> out     */

/* Enqueue one phase of the share on the stream.  One RK4 step is, for
 * stage = 0..3: INVERSE, forward exchange, CROSS, backward exchange,
 * FORWARD; a right-hand side is the same with stage = 4.  GATHER before the
 * first step, SCATTER after the last (in and out are used by these two only;
 * out = canonical share [3][N][N][nkz], every element written, zero outside
 * the retained set).  The exchanges are the caller's; every share must have
 * finished a phase before any share's exchange reads its buffer.
 * Errors: HOT_E_INVALID (phase, stage or pointers; an RK4 plan takes stages
 * 0..3, an RHS plan stage 4), HOT_E_WORKSPACE, HOT_E_HIP. */
int hot_slab_run(hot_plan_t p, int32_t phase, int32_t stage, const void* in, void* out, void* workspace,
                 void* stream);

/* Release the plan's host state (waits for its pending profiling events).
 * NULL is accepted and ignored. */
int hot_destroy(hot_plan_t p);

/* Text for a return code (static storage). */
const char* hot_error_string(int code);

/* HIP error code recorded by the last failing call on this plan, 0 if none. */
int hot_last_hip_error(hot_plan_t p);

/* Per-pass timing.  When enabled, hot_run brackets every kernel launch with
 * HIP events on the run stream.  hot_profile_read waits for those events,
 * writes for each pass id (< max_passes) the summed milliseconds and the
 * number of launches, then clears the record.  Returns the number of pass
 * ids, or a negative error code. */
int hot_profile_enable(hot_plan_t p, int enable);
int hot_profile_read(hot_plan_t p, int32_t max_passes, double* ms, int64_t* launches);

/* Name of pass id (static storage), and the algorithmic HBM bytes one launch
 * of that pass moves for instance i of the plan (each retained input and
 * output value read or written once; 0 if the pass is unused by the op; for
 * "persistent" the passes of a one-step RK4 call). */
const char* hot_pass_name(int32_t pass);
int hot_pass_bytes(hot_plan_t p, int32_t instance, int32_t pass, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* HOT_H */
