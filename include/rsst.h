/*
 * rsst.h -- C ABI of the MI355X (gfx950) explicit time step of the
 * semi-conservative reduced-speed-of-sound technique (RSST) of
 * Iijima, Hotta & Imada, arXiv:1812.04135.
 *
 * One call of rsst_step advances a caller-owned device state by one
 * second-order SSP Runge-Kutta step (Sec. 4.1 "Numerical method") of the
 * finite-volume discretisation of the semi-conservative equations:
 *   - MUSCL reconstruction of the conservative variables with the
 *     monotonized-central limiter;
 *   - local Lax-Friedrichs interface flux with c_tot = |V| + a/xi;
 *   - flux divergence Delta rho, Delta(rho V_i), Delta E   (eq. pvs_dt0);
 *   - Delta P from those increments                       (eq. pvs_dt_dpr,
 *     ideal gas: (de/dP)_rho = 1/(gamma-1), (de/drho)_P = 0; or the
 *     van der Waals gas of rsst_eos);
 *   - the corrected time derivatives of the chosen form:
 *       PVS (eq. pvs_dt), DVS (App. A.1), PMS (App. A.2), DMS (App. A.3),
 *       PD (App. A.4), or plain Euler;
 *   - gravity rho F and rho V.F added after the correction, Delta P
 *     unchanged (App. B);
 *   - CFL time step with Courant number cfl and c_tot (Sec. 4.1, item 1).
 *
 * Conventions
 *   - Status codes: 0 = success, negative = error (see rsst_status).  No
 *     call throws, prints or aborts.
 *   - Device pointers are HIP device allocations owned by the caller unless
 *     stated otherwise.  `stream` is a hipStream_t passed as void*; NULL is
 *     the default stream.
 *   - Fields are structure-of-arrays [nvar][nz][ny][nx], x fastest,
 *     nvar = ndim + 2, variables (rho, rho V_1 .. rho V_ndim, E).  Unused
 *     axes have n = 1.
 *   - A handle is bound to one device and one state size; it is not
 *     thread-safe, and calls on one handle must be ordered on one stream.
 *   - rsst_step enqueues work only: it does not synchronise, allocate or
 *     copy, so a sequence of steps can be captured in a HIP graph.
 */
#ifndef RSST_H
#define RSST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rsst_status {
  RSST_OK = 0,
  RSST_E_ARG = -1,          /* invalid argument or configuration            */
  RSST_E_NOMEM = -2,        /* device allocation failed                     */
  RSST_E_DEVICE = -3,       /* a HIP runtime call failed                    */
  RSST_E_UNSUPPORTED = -4,  /* valid but not supported by this build        */
  RSST_E_NONPHYSICAL = -5,  /* rho <= 0, P <= 0 or a non-finite value seen  */
  RSST_E_SCRATCH = -6       /* state beyond the fixed scratch of
                               rsst_step_noalloc                            */
};

enum rsst_form { RSST_EULER = 0, RSST_PVS = 1, RSST_PMS = 2, RSST_DVS = 3,
                 RSST_DMS = 4, RSST_PD = 5 };
/* Boundary of one side of an axis (Sec. 4.2 periodic, Sec. 4.4 closed
 * free-slip walls).  RSST_REFLECT: mirror ghosts (two layers), the momentum
 * normal to the wall negated; no mass or energy crosses the wall.
 * RSST_REFLECT_HYDRO: the same ghosts, but each ghost's pressure is its
 * mirrored cell's carried to the ghost centre along the external force,
 * P_g = P_k + rho_k g_d (x_g - x_k), which balances gravity at the wall face
 * (no mass crosses the wall; energy does, at O(dx)).  FP64 only, not with
 * the adjoint or the batch, and on axis 0 only with g[0] = 0 (where it is
 * RSST_REFLECT); otherwise RSST_E_UNSUPPORTED. */
enum rsst_bc { RSST_PERIODIC = 0, RSST_REFLECT = 1, RSST_REFLECT_HYDRO = 2 };
enum rsst_prec { RSST_FP64 = 0, RSST_FP32_PERT = 1 };

typedef struct rsst_config {
  int ndim;          /* 1, 2 or 3                                             */
  int n[3];          /* cells per axis (>= 4 on the used axes); axes >= ndim
                        must be 1.  Supported (else RSST_E_UNSUPPORTED): a
                        workgroup holds whole x rows, so n[0] <= 1024 in 1D
                        and 2D and n[0] <= 512 in 3D; a 1D or 2D state is
                        below 2 GiB (32-bit byte offsets); a 3D state may be
                        of any size, with each x-y plane of one variable
                        below 2 GiB.                                          */
  double dx[3];      /* cell widths (> 0) of the used axes                    */
  double gamma;      /* ratio of specific heats, > 1                          */
  double xi;         /* reduction rate of the sound speed, >= 1 (App. A.2)    */
  double cfl;        /* Courant number in (0, 1]; the paper uses 0.4          */
  int dt_rule;       /* 0: dt = cfl / (max c_tot * sum_d 1/dx_d)
                        1: dt = cfl * min_d dx_d / max c_tot                  */
  double g[3];       /* external force per unit mass (App. B)                 */
  int bc_lo[3];      /* rsst_bc of the low side of each axis                  */
  int bc_hi[3];      /* rsst_bc of the high side; a periodic side must face a
                        periodic side                                         */
  int form;          /* rsst_form                                             */
  int prec;          /* rsst_prec.  RSST_FP32_PERT stores U1 = U - U0 in FP32
                        and does all arithmetic in FP64 on U0 + U1            */
  const double* bg;  /* FP32_PERT only: device FP64 background U0, layout
                        [nvar][nbg], caller-owned, must outlive the handle    */
  int bg_axis;       /* -1: U0 uniform (nbg = 1); else the axis it varies on
                        (nbg = n[bg_axis])                                    */
  double t_end;      /* > 0: the CFL step is cut so that t never passes t_end;
                        0: no end time                                        */
  int flags;         /* or of rsst_flag                                       */
  double cmax;       /* > 0: upper limit C_max of the sound speed; xi is then
                        [1 + (a/C_max)^4]^(1/4) of each state's own sound
                        speed a (eq. cx): c_tot of every face state and cell,
                        and f = 1 - 1/xi^2 of every cell's correction.  The
                        field xi is unused.  0: the constant xi.  Not with
                        the batch or the adjoint (RSST_E_UNSUPPORTED).        */
  int eos;           /* rsst_eos: the equation of state of the gas            */
  double eos_a;      /* RSST_EOS_VDW: attraction a >= 0 and co-volume b >= 0  */
  double eos_b;      /* of the van der Waals gas (below); ignored otherwise   */
} rsst_config;

/* Equation of state (Sec. 3.2; the general form enters through the
 * thermodynamic derivatives of eq. pvs_cons_therm in Delta P, eq.
 * pvs_cons_dpr, and through the sound speed in c_tot and the correction).
 *   RSST_EOS_IDEAL: e = P/(gamma-1).
 *   RSST_EOS_VDW:   van der Waals gas with constant specific heat,
 *                   e = (P + a rho^2)(1 - b rho)/(gamma-1) - a rho^2,
 *                   so P = (gamma-1)(e + a rho^2)/(1 - b rho) - a rho^2 and
 *                   a_s^2 = gamma (P + a rho^2)/(rho (1 - b rho)) - 2 a rho.
 *                   e is the internal energy per unit volume, E - rho|V|^2/2.
 *                   FP64 storage with constant xi only (RSST_E_UNSUPPORTED
 *                   with RSST_FP32_PERT, cmax > 0 or RSST_WITH_ADJOINT; the
 *                   batch takes ideal-gas boxes only).  A cell with
 *                   b rho >= 1 is flagged like rho <= 0, one with
 *                   a_s^2 <= 0 like P <= 0. */
enum rsst_eos { RSST_EOS_IDEAL = 0, RSST_EOS_VDW = 1 };

enum rsst_flag {
  RSST_WITH_ADJOINT = 1  /* rsst_init also reserves the workspace of the
                            adjoint calls (FP64 only): on a 2D grid
                            nvar * ncell doubles and three per 16 x 16 tile,
                            else nvar * ncell * (2 ndim + 3) doubles and four
                            per 256 cells.  The adjoint calls of one handle
                            share it: order them on one stream.               */
};

typedef struct rsst_solver* rsst_handle;

/* Validates cfg on the host before touching the device (RSST_E_ARG on any
 * invalid field), then allocates the workspace (stage buffer, scalars, one
 * CFL maximum per stage-kernel workgroup) on the current device and zeroes
 * the scalars and maxima on `stream`, synchronising it before returning (so
 * later calls may use any stream).  t starts at 0.  No allocation happens
 * after this call. */
int rsst_init(const rsst_config* cfg, void* stream, rsst_handle* out);

/* Sets t = t0 and records, on the device, the maxima of c_tot over U from
 * which the next CFL step forms its dt.  rsst_step calls this by itself (t
 * unchanged) on the first CFL step; call it again after writing U from
 * outside.  Every step records the maxima of the state it leaves. */
int rsst_prime(rsst_handle h, const void* U, double t0, void* stream);

/* One SSP-RK2 step of U in place:
 *   U1 = U + dt R(U);   U <- (U + (U1 + dt R(U1))) / 2.
 * U: device array of nvar * ncell doubles (FP64) or floats (FP32_PERT,
 * holding U - U0).  dt_fixed > 0 uses that dt for both stages; dt_fixed <= 0
 * uses the CFL dt of U, computed on the device (no host sync).  Non-physical
 * states are latched on the device and reported by rsst_poll. */
int rsst_step(rsst_handle h, void* U, double dt_fixed, void* stream);

/* One Runge-Kutta stage of rsst_step, for callers that schedule or time the
 * two stages separately.  stage 1: forms the step's dt (a CFL step: from the
 * recorded maxima, cut at t_end) and U1 = U + dt R(U) into the library's
 * stage buffer (U unchanged); stage 2: U <- (U + (U1 + dt R(U1))) / 2,
 * advancing t and recording the maxima of c_tot over the new U.  A stage 2
 * call must follow a stage 1 call on the same U and dt_fixed;
 * rsst_step(h, U, dt, s) is stage 1 then stage 2.  RSST_E_ARG for any other
 * stage number. */
int rsst_stage(rsst_handle h, void* U, int stage, double dt_fixed, void* stream);

/* One rsst_step out of place: U1 = U + dt R(U) into the caller's U1 and
 *   Unext = (U + (U1 + dt R(U1))) / 2,
 * U unchanged.  Same kernels, dt rule and results as rsst_step (Unext holds
 * the bits rsst_step would leave in U; t and the recorded maxima advance the
 * same way).  U1, Unext: device arrays of U's type and size that overlap
 * neither U nor each other (RSST_E_ARG where two of the three pointers are
 * equal).  For callers that keep a trajectory with its stage values, e.g.
 * to hand U1 to rsst_adjoint_step_u1. */
int rsst_step_out(rsst_handle h, const void* U, void* U1, void* Unext, double dt_fixed, void* stream);

/* nsteps calls of rsst_step_out in one call, keeping the trajectory:
 * U_list[n+1] = the step from U_list[n], U1_list[n] its stage value, for
 * n = 0 .. nsteps-1 (U_list: host array of nsteps + 1 device pointers,
 * U_list[0] the start state, read only; U1_list: nsteps).  Same results as
 * the separate calls; every launch on `stream` from this call.  RSST_E_ARG
 * for a NULL entry or nsteps < 0; a pair of equal pointers within one step
 * is refused as rsst_step_out refuses it, after the steps before it ran. */
int rsst_steps_out(rsst_handle h, void* const* U_list, void* const* U1_list, int nsteps, double dt_fixed,
                   void* stream);

/* nsteps calls of rsst_step, with the same results.  A 1D grid runs as one
 * workgroup, so for ndim = 1 all nsteps steps are one launch (both stages,
 * the CFL maximum and the next dt of every step inside it, U written once at
 * the end; the stage buffer's contents are then unspecified); there, with a
 * CFL step and t_end > 0, the steps left once t reaches t_end (dt = 0, which
 * leave U unchanged) are skipped. */
int rsst_steps(rsst_handle h, void* U, int nsteps, double dt_fixed, void* stream);

/* Returns the time t and the dt the next CFL step will use (Sec. 4.1, the
 * Courant condition).  The dt is formed on the device, on the stream, by the
 * grid maximum and dt code of stage 1 over the recorded per-workgroup maxima,
 * so it has the same bits; it is 0 before any state has been recorded.
 * Launches one small kernel, then synchronises the stream. */
int rsst_get_time(rsst_handle h, double* t, double* dt_next, void* stream);

/* FP64 diagnostics of U, summed over cells in a fixed order (deterministic):
 * out[0..7] = (sum rho, sum m1, sum m2, sum m3, sum E, sum |m|^2/(2 rho),
 *              max |V|, max xi |V| / a), sums times the cell volume.  The
 * sums are the conserved totals of Sec. 5 (which forms conserve mass,
 * momentum or energy) and the kinetic energy; max xi |V| / a is the
 * effective Mach number whose bound Sec. 4.3 discusses (with C_max, xi of
 * each cell's own sound speed, eq. cx).  Synchronises the stream. */
int rsst_diag(rsst_handle h, const void* U, double out[8], void* stream);

/* Synchronises, copies the non-physical flags seen since the last poll into
 * *flags (bit 0: rho <= 0, bit 1: P <= 0, bit 2: non-finite), clears them,
 * and returns RSST_E_NONPHYSICAL if any was set. */
int rsst_poll(rsst_handle h, uint32_t* flags);

/* Frees the workspace.  The caller's arrays are untouched. */
int rsst_destroy(rsst_handle h);

/* ---- One step that allocates nothing --------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * step as rsst_step on a fresh handle (the same kernels, so the same bits):
 * U advances by one SSP-RK2 step from t = 0 with dt_fixed > 0, or with the
 * CFL dt of U formed on the device when dt_fixed <= 0.  No handle: cfg is
 * validated on the host as by rsst_init (RSST_E_ARG), and RSST_WITH_ADJOINT
 * or t_end != 0 give RSST_E_UNSUPPORTED (the time and the maxima are not
 * kept between calls).  U: caller-owned device state as for rsst_step.
 * flags: NULL, or a caller-owned device word that receives the step's
 * non-physical flags (as rsst_poll's).  Scratch (device scalars, CFL maxima
 * and the stage buffer U1) is a fixed 64 MiB device array of the library,
 * held by each device it runs on until the process ends.  It takes a copy
 * of the state, nvar * ncell * sizeof(value) bytes, plus 256 B of scalars
 * and 8 B per stage-kernel workgroup (each part rounded up to 256 B); a
 * configuration that needs more than 64 MiB (a 2D 1024^2 FP64 state needs
 * 32 MiB, a 3D 128^3 FP32 perturbation 40 MiB) gives RSST_E_SCRATCH before
 * any device call.  Calls no allocating routine; enqueues only
 * (graph-capturable).
 * All calls on one device share that scratch: calls that overlap on one
 * device race, so order them on one stream. */
int rsst_step_noalloc(const rsst_config* cfg, void* U, double dt_fixed, uint32_t* flags, void* stream);

/* ---- Adjoint -------------------------------------------------------------
 * Discrete adjoint of one rsst_step of fixed dt (dt frozen: the CFL rule is
 * not differentiated).  The step is U' = (U + U1 + dt R(U1)) / 2 with
 * U1 = U + dt R(U), R the semi-discrete operator of Sec. 4.1 with the
 * correction of the configured form (eq. pvs_dt, App. A) and gravity
 * (App. B).  Given lam = dJ/dU' it computes, in place,
 *   lam <- (dU'/dU)^T lam        and        *dJdxi += (dU'/dxi)^T lam,
 * with the branch-frozen derivatives of the primal values: the MC limiter
 * is 0 where l r <= 0, else it follows the first minimum of
 * (|l+r|/2, 2|l|, 2|r|); the LLF speed is c_L where c_L >= c_R, else c_R;
 * d|V| = 0 at V = 0.
 * h: an FP64 handle made with flags & RSST_WITH_ADJOINT (else
 * RSST_E_UNSUPPORTED).  U: device FP64 state at the start of the step (read
 * only).  lam: device FP64 [nvar][ncell], in/out.  dt > 0: the dt the
 * forward step used.  dJdxi: device double, accumulated.  U1 is recomputed
 * in the handle's stage buffer, so the call must not fall between the two
 * stages of a forward rsst_stage pair on the same handle.  Enqueues only. */
int rsst_adjoint_step(rsst_handle h, const void* U, double* lam, double dt, double* dJdxi, void* stream);

/* rsst_adjoint_step with the step's stage value given: U1 = U + dt R(U) as
 * rsst_step_out left it for this U and dt (device FP64, read only), so it is
 * not recomputed and the handle's stage buffer is not touched.  Same results
 * as rsst_adjoint_step, bit for bit. */
int rsst_adjoint_step_u1(rsst_handle h, const void* U, const void* U1, double* lam, double dt, double* dJdxi,
                         void* stream);

/* The adjoint of nsteps fixed-dt steps over a trajectory kept by the caller:
 * for n = nsteps-1 down to 0, the rsst_adjoint_step_u1 of the step from
 * U_list[n] with stage value U1_list[n] (both as rsst_step_out left them),
 * lam in place; then *dJdxi += the run's dJ/dxi.  U_list, U1_list: host
 * arrays of nsteps device pointers (FP64); U1_list may be NULL (each stage
 * value is then recomputed, as rsst_adjoint_step does).  lam leaves with the
 * bits of nsteps rsst_adjoint_step_u1 calls; on a 2D grid dJ/dxi is summed
 * per tile over the run and folded once at the end (the same value to
 * rounding, not the same bits as per-call folds).  All launches on `stream`
 * from this one call, so the device runs the steps back to back.
 * RSST_E_ARG for a NULL entry, nsteps < 0 or dt <= 0. */
int rsst_adjoint_run(rsst_handle h, const void* const* U_list, const void* const* U1_list, int nsteps, double* lam,
                     double dt, double* dJdxi, void* stream);

/* ---- Batched boxes ------------------------------------------------------
 * Many independent 2D boxes (each with its own size, xi, gravity, boundaries
 * and background) advanced together by one persistent kernel per run; the
 * run (counter reset, per-box CFL prime, persistent kernel) is captured in a
 * HIP graph on first use and replayed while U_all, nsteps and the strip rows
 * are unchanged.  Each box takes its own CFL dt every step, from the
 * maximum c_tot over that box only.  Same numerics as rsst_step per box.
 * This build: ndim = 2, n[0] <= 256, one form and one prec for all boxes,
 * t_end = 0; FP32_PERT backgrounds vary along y (bg_axis = 1) or not (-1). */
typedef struct rsst_batch_s* rsst_batch;

/* boxes[nbox]: per-box configurations (validated on the host).  offsets[b]:
 * element offset of box b's [nvar][ny][nx] block inside the caller's U_all
 * array (FP64, or FP32 for FP32_PERT); blocks must not overlap.  max_steps:
 * the largest nsteps a run will ask for (sizes the per-step counters).
 * Allocates the stage buffer and the queue state; nothing after this call
 * except the graph of a run. */
int rsst_batch_init(const rsst_config* boxes, int nbox, const int64_t* offsets, int max_steps,
                    void* stream, rsst_batch* out);

/* Rows per strip of the march for boxes whose rows span 1, 2, 3 and 4 waves
 * (nx in 1..64, 65..128, 129..192, 193..256); each in [8, 256].  Takes
 * effect at the next run (re-captures the graph).  Default 16. */
int rsst_batch_set_tiles(rsst_batch h, const int strip_rows[4]);
int rsst_batch_get_tiles(rsst_batch h, int strip_rows[4]);

/* The work items a run would execute for these boxes and strip rows, on the
 * host only (no device call): one row of RSST_BATCH_PLAN_COLS ints per
 * item, (box, block, first row, end row, ndep, dep[0..7]) where dep lists
 * the blocks of the same box (-1 padded) whose stencil reads this block's
 * rows or whose rows this block's stencil reads (two cells in y through the
 * boundary rule); an item runs only after those blocks finished the
 * previous stage.  Writes at most cap rows to table and the item count to
 * *nitem (call with cap = 0 to size). */
#define RSST_BATCH_PLAN_COLS 13
int rsst_batch_plan(const rsst_config* boxes, int nbox, const int strip_rows[4], int* table, int cap,
                    int* nitem);

/* nsteps SSP-RK2 steps of every box of U_all, in place, enqueued on stream.
 * 1 <= nsteps <= max_steps.  The first call (or a call with a different
 * U_all, nsteps or strip rows) synchronises the stream, uploads the tables
 * and captures the graph; later calls only launch it. */
int rsst_batch_run(rsst_batch h, void* U_all, int nsteps, void* stream);

/* Synchronises, then copies the time reached by every box into t[nbox]. */
int rsst_batch_times(rsst_batch h, double* t, void* stream);

/* As rsst_poll, for the batch, with one more flag: bit 3 (8) is set when a
 * work item gave up waiting for a dependency (see rsst_batch_set_wait_limit);
 * then the call returns RSST_E_DEVICE and the run's results are invalid. */
int rsst_batch_poll(rsst_batch h, uint32_t* flags);

/* Longest time, in seconds (0 to 3600; default 10), that a work item of a
 * run waits for the items it depends on.  Past it the item is skipped
 * (nothing computed or stored, but marked done, so every workgroup drains
 * and the kernel ends) and the run is flagged for rsst_batch_poll: a
 * dependency that never arrives ends the run with an error instead of a
 * hang.  Takes effect at the next run.  A limit of 0 gives up on any wait
 * that is not satisfied at once, which tests of the error path use. */
int rsst_batch_set_wait_limit(rsst_batch h, double seconds);

/* Synchronises, then sets the time of every box to t[nbox] (host array) and
 * the latched non-physical flags to `flags` (bits as rsst_poll reports
 * them).  For callers that advance the batch on scratch data and restore the
 * record afterwards, as the strip-row autotuner does. */
int rsst_batch_set_times(rsst_batch h, const double* t, uint32_t flags, void* stream);

int rsst_batch_destroy(rsst_batch h);

/* Static string for a status code. */
const char* rsst_strerror(int status);

/* Library build identifier (kernel revision), for logs. */
const char* rsst_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RSST_H */
