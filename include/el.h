/*
 * el.h -- C ABI of the elastic PACT operator pair on one AMD Instinct MI355X (gfx950).
 *
 * The library applies the discrete forward operator H and its exact adjoint
 * H^T of Mitsuhashi et al., "A forward-adjoint operator pair based on the
 * elastic wave equation for use in transcranial photoacoustic computed
 * tomography":
 *
 *   p_hat = H p0      H   = M' T'_{M-1} ... T'_1 T'_0      (Appendix, eq. HPML)
 *   p_adj = H^T y     H^T = T'_0^T ... T'_{M-1}^T M'^T     (Appendix, eq. adjHPML)
 *
 * where each T'_m advances the 4th-order staggered-grid velocity-stress FDTD
 * scheme of the lossy heterogeneous elastic wave equation (Sec. 2.2, eq. it;
 * Appendix, C-PML memory-variable updates) by one step dt, T'_0 injects the
 * initial pressure as the isotropic stress -p0/3 (Sec. 2.1, eq. Ini; Sec. 3,
 * eq. initialp0) and M' samples the pressure -(s11+s22+s33) at the
 * transducers by trilinear interpolation (Sec. 3, eq. interpgrid).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid: nx*ny*nz cells, x fastest: cell (i,j,k) is element i + nx*(j + ny*k)
 *    of every volume array.  Normal stresses, lambda, mu, p0 sit on cell
 *    (i,j,k); u1, u2, u3 at (i+1/2,j,k), (i,j+1/2,k), (i,j,k+1/2); s12, s13,
 *    s23 at (i+1/2,j+1/2,k), (i+1/2,j,k+1/2), (i,j+1/2,k+1/2).  Fields are
 *    zero outside the grid.
 *  - The C-PML occupies the outer npml cells of each face (inside the grid).
 *  - Time: nsteps = M samples t_m = m dt, m = 0..M-1, i.e. M-1 updates.
 *  - Traces are double precision, time-major: traces[m*L + l].
 *  - Units are SI: Pa, kg/m^3, 1/s (velocity damping rate of the diffusive
 *    absorption model, Sec. 2.1 eq. subeq1), metres, seconds.
 *  - Memory: every pointer marked (device) is device memory of the GPU that
 *    is current when the call is made; (host) is ordinary host memory.  The
 *    caller owns every buffer, the workspace included; the library never
 *    allocates device memory.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  Operations are asynchronous with respect to the host unless
 *    stated otherwise; successive operations on one plan are ordered even
 *    when issued on different streams.
 *  - Errors: every call returns EL_OK (0) or a negative el_status; the detail
 *    of the last failure on the calling thread is returned by el_last_error().
 *    Argument checks run on the host before anything is enqueued, so a
 *    rejected call leaves device memory untouched.  No C++ exception crosses
 *    this interface.
 */
#ifndef EL_H
#define EL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t el_status;
#define EL_OK         0
#define EL_EINVAL    -1   /* malformed argument, bad material value, null pointer          */
#define EL_EUNSTABLE -2   /* CFL above 6/(7 sqrt 3) or dt*alpha outside [0,1)               */
#define EL_ERANGE    -3   /* a receiver outside [0, n-1]*dx on some axis                    */
#define EL_ENOMEM    -4   /* workspace smaller than el_plan_bytes() says                    */
#define EL_EDEVICE   -5   /* a HIP runtime call failed                                      */
#define EL_EBUSY     -6   /* every executor or group slot is in use                         */

#define EL_F32 0          /* fields, stencils, p0 and p_adj in float  */
#define EL_F64 1          /* fields, stencils, p0 and p_adj in double */

/*
 * Frequency-dependent absorption.  The paper's absorption is diffusive: the
 * velocity is damped at a rate alpha that does not depend on frequency
 * (Sec. 2.1, eq. subeq1); its conclusion (Sec. 8) names a frequency-dependent
 * attenuation model as the next step.  With nmech > 0 relaxation mechanisms
 * join the damping term:
 *
 *   d/dt u + alpha u + sum_l beta_l (u - zeta_l) = div(sigma) / rho,
 *   d/dt zeta_l = omega_l (u - zeta_l),   beta_l = weight[l] * alpha_r,
 *
 * i.e. a damping rate a(w) = alpha + sum_l beta_l i w / (omega_l + i w) that
 * rises with frequency w.  alpha_r is a cell map (el_plan_create), averaged
 * at the velocity points like alpha.  Discretely, every step's velocity
 * update is followed by the pointwise sub-update
 *   u' = (u + dt sum_l beta_l zeta_l) / (1 + dt sum_l beta_l),
 *   zeta_l' = c_l zeta_l + (1 - c_l) u',   c_l = exp(-omega_l dt),
 * and the adjoint applies its transpose at the mirrored place, so H^T stays
 * the exact transpose.  nmech = 0 is the paper's diffusive model.
 */
#define EL_MAX_MECH 4
typedef struct {
    int32_t nmech;              /* 0 .. EL_MAX_MECH relaxation mechanisms                      */
    double  omega[EL_MAX_MECH]; /* their angular frequencies omega_l > 0 (rad/s)               */
    double  weight[EL_MAX_MECH];/* their weights w_l >= 0                                      */
} el_relaxation;

typedef struct {
    int32_t nx, ny, nz;   /* cells per axis, C-PML included; each >= 4 and >= 2*npml + 2      */
    double  dx;           /* grid spacing (m), the same on every axis                          */
    double  dt;           /* time step (s)                                                     */
    int32_t nsteps;       /* M >= 1 trace samples (M-1 updates)                                */
    int32_t npml;         /* C-PML thickness in cells on every face; 0 = no layer              */
    double  pml_R;        /* target reflection of the layer; <= 0 selects 1e-3                 */
    double  pml_npower;   /* damping profile power; <= 0 selects 2                             */
    double  pml_f0;       /* frequency (Hz) of the profile's beta = pi f0 (1 - xi);            */
                          /*   <= 0 selects 1500 / (8 dx)                                      */
    int32_t precision;    /* EL_F32 or EL_F64                                                  */
    el_relaxation relax;  /* frequency-dependent absorption; all zero = none                  */
} el_grid;

typedef struct el_plan_* el_plan;

/* Library version string (static storage). */
const char *el_version(void);

/* Name of a status code (static storage). */
const char *el_status_string(el_status status);

/* Detail of the last failed call on the calling thread ("" if none). */
const char *el_last_error(void);

/*
 * Host-only checks of a grid and a receiver set: sizes, spacing, PML
 * thickness, precision, that every array the kernels address (a padded
 * volume, a C-PML memory-variable slab of 2 (npml + 7) planes) stays below
 * 4 GiB, the relaxation mechanisms (nmech in 0..EL_MAX_MECH, every omega_l
 * > 0 and weight w_l >= 0 finite), and that every receiver lies in
 * [0, n-1]*dx (up to 1e-9 cells of rounding; such receivers are clamped
 * onto the box).
 * rec_xyz (host): nrec x 3 doubles, metres from the centre of cell (0,0,0),
 * columns x, y, z.  nrec may be 0 (rec_xyz may then be NULL).
 * Returns EL_EINVAL or EL_ERANGE on failure.  Touches no device.
 */
el_status el_grid_check(const el_grid *grid, const double *rec_xyz, int32_t nrec);

/*
 * Device workspace bytes a plan of this grid and receiver count needs
 * (fields, material maps, C-PML boundary slabs, PML tables, receiver
 * tables, reduction scratch; with relaxation mechanisms the strength map and
 * room for a point list and its memory variables of up to three velocity
 * points per cell).  Host-only; *bytes is written on success.
 */
el_status el_plan_bytes(const el_grid *grid, int32_t nrec, size_t *bytes);

/*
 * Build a plan: validate, copy the material maps into the workspace,
 * compute the C-PML profiles (Appendix A.1-A.2, kappa = 1) and the
 * trilinear receiver tables (Sec. 3, eq. interpgrid).
 *   lambda, mu, rho, alpha (device): N = nx*ny*nz floats each, cell values
 *       in Pa, Pa, kg/m^3, 1/s.  Checked on the device: rho > 0, mu >= 0,
 *       lambda + 2 mu > 0, 3 lambda + 2 mu > 0 (a positive bulk modulus,
 *       Sec. 2.1), 0 <= dt*alpha < 1, all finite (EL_EINVAL /
 *       EL_EUNSTABLE), and max sqrt((lambda+2mu)/rho) dt/dx <= 6/(7 sqrt 3)
 *       (EL_EUNSTABLE).  They may be freed once this call returns.
 *   alpha_r (device): with grid->relax.nmech > 0, N floats, the strength of
 *       the relaxation mechanisms in 1/s (see el_relaxation); finite, >= 0,
 *       and 0 on every cell within npml + 2 cells of a face (the C-PML
 *       layers and their neighbours: the adjoint's layer variables are
 *       updated inside the velocity pass, before the transposed relaxation),
 *       else EL_EINVAL.  Ignored (may be NULL) when nmech = 0.
 *   rec_xyz (host): nrec x 3 doubles as in el_grid_check().
 *   workspace (device): at least el_plan_bytes() bytes, 256-byte aligned,
 *       owned by the caller, valid until el_plan_destroy().
 * Synchronous: returns after the stream has drained the setup work.
 * On success *out receives the plan; on failure *out is NULL.
 */
el_status el_plan_create(el_plan *out, const el_grid *grid,
                         const float *lambda, const float *mu, const float *rho, const float *alpha,
                         const float *alpha_r, const double *rec_xyz, int32_t nrec,
                         void *workspace, size_t workspace_bytes, void *stream);

/* Release the plan's host state.  The workspace stays the caller's. */
el_status el_plan_destroy(el_plan plan);

/*
 * traces = H p0  (Appendix, eq. STforHPML).
 *   p0 (device): N elements, float for EL_F32 plans, double for EL_F64 plans.
 *   traces (device): nsteps x nrec doubles, time-major, fully overwritten.
 * Asynchronous on `stream`.
 */
el_status el_forward(el_plan plan, const void *p0, double *traces, void *stream);

/*
 * traces = H p0 as el_forward (the same kernels, bit for bit the same traces
 * and final state), and the modified energy of the leapfrog recursion
 * (Sec. 2.2, eq. it) at every `every`-th time level m = 0, every, 2 every,
 * ... <= nsteps - 2, accumulated in double on the device:
 *
 *   E_m = 1/2 sum_c sum_cells rho_c u^c_{m-1/2} u^c_{m+1/2} + 1/2 sigma_m^T C^+ sigma_m
 *
 * with u_{-1/2} = 0, rho_c the staggered density of the update, and
 * sigma^T C^+ sigma = (tr s)^2 / (9K) + |dev s|^2 / (2 mu) at normal points
 * (K = lambda + 2 mu / 3; the second term only where mu > 0) plus
 * s_ij^2 / mu_ij at shear points (only where the harmonic-mean edge modulus
 * mu_ij is nonzero).  The scheme is skew with a symmetric stiffness, so with
 * alpha = 0 and npml = 0 E_m stays constant up to rounding; absorption and
 * the C-PML make it decay.  The C-PML memory variables are not part of E_m.
 *   every: >= 1.
 *   energy (device): ceil((nsteps - 1) / every) doubles (none when
 *       nsteps = 1; energy may then be NULL), fully overwritten in order of m.
 * Deterministic (fixed reduction order).  Asynchronous on `stream`.
 * Errors: EL_EINVAL for a NULL plan, p0, traces (nrec > 0) or energy,
 * every < 1, or a plan with relaxation mechanisms (their memory variables
 * hold energy this sum does not count).
 */
el_status el_forward_energy(el_plan plan, const void *p0, double *traces, int32_t every, double *energy,
                            void *stream);

/*
 * p_adj = H^T y, by the backward recursion v_{m-1} = Theta^T y_{m-1} + W'^T v_m
 * with v_{M-1} = Theta^T y_{M-1} and p_adj = tau'^T v_0 (Sec. 4, eq. Adjup;
 * Appendix eq. AdjupPML read with index m-1).
 *   y (device): nsteps x nrec doubles, time-major.
 *   p_adj (device): N elements of the plan's precision, fully overwritten.
 * Asynchronous on `stream`.
 */
el_status el_adjoint(el_plan plan, const double *y, void *p_adj, void *stream);

/*
 * *out = <a, b> accumulated in double (the inner products of the paper's
 * dot-product test, Sec. 5).  space 0: a, b (device) hold N elements of the
 * plan's precision; space 1: a, b (device) hold nsteps*nrec doubles.
 * out (device): one double.  Deterministic (fixed reduction order).
 * Asynchronous on `stream`.
 */
el_status el_dot_f64(el_plan plan, int32_t space, const void *a, const void *b, double *out, void *stream);

/*
 * *out = <a, b> accumulated in double, as el_dot_f64 computes it (the same
 * kernels and reduction order, so the same double), without a plan and
 * without any device memory from the caller beyond a, b and out.  For
 * callers that cannot allocate device memory: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The library calls
 * no allocating routine here; the partial sums live in a static device
 * array of the library (8 KiB per GPU, kept until the process ends), whose
 * address is looked up on the first call on each device.
 *   precision: EL_F32 (a, b hold floats) or EL_F64 (doubles).
 *   n: element count, 0 .. 2^40 (the partial sums are a fixed 1024 doubles
 *      whatever n is; a, b may be NULL when n = 0, which gives 0).
 *   a, b, out (device): n elements each; one double.
 * Every call on a GPU shares that GPU's array: calls that overlap in time
 * on one GPU (different streams, or different host threads) race and may
 * return wrong sums; calls ordered on one stream do not.  Nothing in the
 * array needs clearing: each call writes every partial sum before reading it.
 * Asynchronous on `stream`.  Errors: EL_EINVAL for a precision other than
 * EL_F32 / EL_F64, n outside 0 .. 2^40, or a NULL out (or a, b with n > 0);
 * EL_EDEVICE if the array's address cannot be obtained.
 */
el_status el_dot_f64_noalloc(int32_t precision, int64_t n, const void *a, const void *b, double *out, void *stream);

/*
 * Transducer response.  The recorded signal is the pressure at the
 * transducer convolved in time with the transducer's electrical impulse
 * response (Sec. 2.3, the imaging model with the transducer's temporal
 * response; the measured-data studies deconvolve it).  With one causal kernel
 * h[0..nh-1] for every receiver, the operator E on traces [M][L] and its
 * adjoint (a correlation) are
 *   transpose 0:  out[m][l] = sum_{k=0}^{min(m, nh-1)}     h[k] in[m-k][l]
 *   transpose 1:  out[m][l] = sum_{k=0}^{min(M-1-m, nh-1)} h[k] in[m+k][l]
 * so E H is the imaging model with the response and H^T E^T its adjoint.
 *   h (device): nh doubles.  in, out (device): nsteps * nrec doubles,
 *   time-major, not overlapping.  No plan is needed.
 * Asynchronous on `stream`.  Errors: EL_EINVAL for NULL pointers, nh < 1,
 * nsteps < 1, nrec < 0, transpose outside 0..1, overlapping in/out.
 */
el_status el_eir_apply(const double *h, int32_t nh, const double *in, double *out, int32_t nsteps, int32_t nrec,
                       int32_t transpose, void *stream);

/*
 * Device pointer and element count of one of the plan's wavefield arrays,
 * for inspection after an operation has completed: id 0..2 = u1, u2, u3;
 * 3..8 = s11, s22, s33, s23, s13, s12 (elements of the plan's precision).
 * The arrays are stored padded (see el_plan_layout); *count is the padded
 * element count.  After el_forward they hold u_{M-3/2} and sigma_{M-1};
 * after el_adjoint they hold the adjoint state of step 0 in the variables
 * r = Q^{-1} q (ids 0..2, the velocity adjoint divided by the staggered
 * density) and w = C s (ids 3..8, the Voigt stiffness applied to the stress
 * adjoint).
 */
el_status el_plan_field(el_plan plan, int32_t id, void **ptr, size_t *count);

/*
 * Padded layout of the wavefield arrays: cell (i, j, k) is element
 * origin + k * plane_pitch + j * row_pitch + i.  The padding holds zeros.
 */
el_status el_plan_layout(el_plan plan, int64_t *row_pitch, int64_t *plane_pitch, int64_t *origin);

/*
 * Extent of the relaxation sub-update (el_relaxation): the stencil tiles
 * holding a velocity point with beta > 0, their cells, and the (cell,
 * component) velocity points with beta > 0, the list it updates (built once
 * by el_plan_create).  All zero for a plan without relaxation mechanisms.
 * Any pointer may be NULL.  Host-only.
 */
el_status el_plan_relaxation(el_plan plan, int64_t *tiles, int64_t *cells, int64_t *points);

/* Number of cells N, receivers L and trace samples M of a plan. */
el_status el_plan_sizes(el_plan plan, int64_t *ncells, int32_t *nrec, int32_t *nsteps);

/*
 * Fluid tiles.  Where the shear modulus is zero (the fluid limit of the
 * elastic equations, Sec. 2.1) the stress update keeps the three normal
 * stresses equal and the shear stresses at zero; the same holds for the
 * adjoint state w = C s.  At plan creation every stencil tile (64 x 4 cells
 * by a chunk of z planes) whose cells, and the cells within two of them,
 * all have mu = 0 is marked, and the stencil passes update such tiles from
 * the normal stress s11 alone, with only the diagonal C-PML memory
 * variables: fewer bytes, the same results.  The shear stresses are not
 * written.  s22 and s33 equal s11 there; s22 is stored only on the two
 * rows along a y face, and s33 only on the two planes along a z face, shared
 * with a tile that takes the general update (whose taps read them there).
 * The receiver gather takes 3 s11 as the trace of a cell in a fluid tile,
 * and at the end of every operation one pass sets s22 = s33 = s11 on all
 * fluid tiles, so el_plan_field shows the full state.  A fluid tile whose
 * lambda, rho and alpha are each one value over that box (a homogeneous
 * coupling medium such as the water of Sec. 7) takes the three values from
 * a per-tile table instead of the maps, again with the same results.
 * Inside the other tiles, every column of 1 x 1 cells by the chunk whose
 * cells within two have mu = 0 is marked too and takes the fluid update,
 * storing all three normal stresses: a wavefront (32 x 2 cells of the tile)
 * of such columns runs the fluid loop, and in a wavefront that also holds
 * other columns the fluid lanes run the general loop without the loads they
 * do not need (shear stresses, moduli).
 * A column whose box holds the tile's reference medium (that of its first
 * fluid column) takes it from the table as well.
 */
typedef struct el_fluid_stats {
    int64_t tiles;           /* tiles that take the fluid update                   */
    int64_t cells;           /* cells that take it (fluid tiles and columns)       */
    int64_t layer_cells;     /* sum over the three axes of those cells in the      */
                             /* axis's C-PML layers (depth > 0): only the diagonal */
                             /* memory variable is carried there                   */
    int64_t skipped_stores;  /* s22 and s33 stores (cell, component pairs) one     */
                             /* stress pass leaves out                             */
    int64_t uniform_cells;   /* fluid-update cells whose lambda, rho, alpha come   */
                             /* from the per-tile table: uniform fluid tiles, and  */
                             /* fluid columns of their tile's reference medium     */
    int64_t column_cells;    /* cells of fluid columns inside other tiles          */
} el_fluid_stats;

/*
 *   enable: 1 use the fluid update where it applies (the default), 0 never,
 *           -1 keep the current setting.  A change waits for the plan's
 *           previous operation (host-blocking).
 *   *stats (host, may be NULL): the counts under the resulting setting (all
 *           zero when the fluid update is off).
 * Errors: EL_EINVAL for a NULL plan or an enable outside -1..1.
 */
el_status el_plan_fluid_path(el_plan plan, int32_t enable, el_fluid_stats *stats);

/* Kernel kinds reported by el_plan_kernel_time(). */
#define EL_K_VELOCITY     0   /* forward velocity pass (+ phi slabs; it also   */
                              /* gathers the previous trace row)               */
#define EL_K_STRESS       1   /* forward stress pass (+ psi slabs)             */
#define EL_K_ADJ_VELOCITY 2   /* adjoint pass producing the velocity adjoint   */
#define EL_K_ADJ_STRESS   3   /* adjoint pass producing the stress adjoint     */
                              /* (it also scatters the next trace row)         */
#define EL_K_GATHER       4   /* receiver gather of the last trace row         */
#define EL_K_SCATTER      5   /* receiver scatter of the last trace row        */
                              /* (adjoint; the first thing H^T does)           */
#define EL_K_RELAX        6   /* relaxation sub-update (forward) or its        */
                              /* transpose (adjoint), plans with nmech > 0     */
#define EL_K_COUNT        7

/*
 * Benchmark instrumentation.  With every = n >= 1, the kernel launches of the
 * time loops of later el_forward / el_adjoint calls that belong to time steps
 * m with m mod n = 0 (n = 1: every launch) are each bracketed by a pair of
 * HIP events recorded on that call's stream; every = 0 stops recording.  An
 * event between two kernels costs each a few microseconds of issue gap, so a
 * sample of the steps keeps the timed loop close to its untimed speed.
 * el_plan_kernel_time() waits for the recorded events, returns how many
 * launches of one kind were recorded and their summed duration in ms, and
 * clears the record of that kind.  Host-blocking; not for production loops.
 * Errors: EL_EINVAL for a NULL plan or a negative every.
 */
el_status el_plan_timing(el_plan plan, int32_t every);
el_status el_plan_kernel_time(el_plan plan, int32_t kind, int64_t *launches, double *total_ms);

/*
 * Executor: many operations in flight at once (serving).
 *
 * An executor owns `max_slots` slots, each with its own HIP stream (default
 * priority).  el_exec_start enqueues a whole operation of a plan on a free
 * slot and returns at once: the initial state, then the time loop as replays
 * of a captured graph of `chunk_steps` steps (a device step counter selects
 * the trace row, so one graph serves every chunk), then the extraction of the
 * adjoint.  Operations on different slots overlap on the device.  With a
 * replay limit (el_exec_set_ahead) a slot holds at most that many replays in
 * flight and el_exec_poll / el_exec_pump / el_exec_wait enqueue the rest as
 * earlier ones complete, so the host must keep calling them.  Results are
 * identical to el_forward / el_adjoint on the same plan.  The operation is
 * ordered after the plan's previous operation; the plan must not be used
 * again, nor its buffers released, before el_exec_poll reports completion.
 * The buffers (plan workspace, in, out) are the caller's, as for el_forward.
 */
#define EL_OP_FORWARD 0   /* in: p0 (plan precision, N), out: traces (double, M x L) */
#define EL_OP_ADJOINT 1   /* in: y (double, M x L), out: p_adj (plan precision, N)  */

typedef struct el_exec_ *el_exec;

/* Create an executor on the current device.  max_slots in 1..64, chunk_steps >= 1. */
el_status el_exec_create(el_exec *out, int32_t max_slots, int32_t chunk_steps);

/* Enqueue what a replay limit has held back, wait for every slot, then release the executor. */
el_status el_exec_destroy(el_exec ex);

/*
 * Start `op` on a free slot; *slot receives its index.  EL_EBUSY if all slots
 * are busy.  The operation runs after all work enqueued so far on `stream`
 * (the caller's stream that writes `in` or last used `out`; NULL = the null
 * stream) and after the plan's previous operation.
 */
el_status el_exec_start(el_exec ex, el_plan plan, int32_t op, const void *in, void *out, void *stream,
                        int32_t *slot);

/* Non-blocking: *done = 1 once the slot's operation has completed (the slot is then free). */
el_status el_exec_poll(el_exec ex, int32_t slot, int32_t *done);

/* Block until the slot's operation has completed (the slot is then free). */
el_status el_exec_wait(el_exec ex, int32_t slot);

/* Number of slots and how many are running an operation. */
el_status el_exec_slots(el_exec ex, int32_t *total, int32_t *busy);

/*
 * Replays of the step graph each slot keeps in flight: 0 (the default) enqueues
 * an operation whole at el_exec_start; r in 1..1024 enqueues r replays there and
 * the rest from el_exec_poll / el_exec_pump / el_exec_wait as earlier replays
 * complete, which bounds how much of one slot's work is queued ahead of other
 * streams.  EL_EBUSY while a slot is running; EL_EINVAL for r outside 0..1024;
 * EL_EDEVICE if the replay events cannot be created (the executor is then unlimited).
 */
el_status el_exec_set_ahead(el_exec ex, int32_t replays);

/* Non-blocking: enqueue what the replay limit allows on every running slot. */
el_status el_exec_pump(el_exec ex);

/*
 * Group: grouped time stepping of many operations (serving).
 *
 * A group holds up to `max_members` operations of one precision, each on its
 * own plan (grids, media, step counts and receivers may differ).  el_group_run
 * advances every running member by one time step per tick, the same step as
 * el_forward / el_adjoint take (Sec. 2.2 for H, its transpose for H^T): one
 * velocity launch and one stress launch (which, for adjoint members, also adds
 * Theta^T of the trace row) serve up to four members at once, their tiles side
 * by side in one grid, so that small grids share the device.  Members join (el_group_add) and leave (after their
 * last step, or el_group_remove) between ticks; nothing is captured, the
 * launch arguments are rebuilt each tick.  A member's result is bitwise that
 * of el_forward / el_adjoint on its plan.
 *
 * All work runs on the group's own stream (default priority) and returns at
 * once.  A member's plan must not be used elsewhere, nor its buffers
 * released, before el_group_poll reports it done.  Calls on one group must not
 * overlap (one host thread at a time).
 */
typedef struct el_group_ *el_group;

/* Create a group on the current device.  max_members in 1..64; precision
 * EL_F32 or EL_F64 (every member's plan must have it).  EL_EDEVICE if the
 * stream or events cannot be created. */
el_status el_group_create(el_group *out, int32_t max_members, int32_t precision);

/* Wait for the group's stream, then release the group (members' buffers are
 * the caller's). */
el_status el_group_destroy(el_group g);

/*
 * Add `op` on `plan` as a member; *slot receives its index.  Enqueues the
 * initial state (Sec. 2.2: zero fields, then p0 injected through tau' for the
 * forward, Theta^T of the last trace row for the adjoint) after all work
 * enqueued so far on `stream` (the caller's stream that writes `in`; NULL =
 * the null stream) and after the plan's previous operation.  in/out as for
 * el_exec_start.  A plan with nsteps = 1 finishes here.  EL_EBUSY if every
 * slot is used; EL_EINVAL for a bad op, NULL buffers, a plan of another
 * precision or device, or a plan that is already a member.
 */
el_status el_group_add(el_group g, el_plan plan, int32_t op, const void *in, void *out, void *stream,
                       int32_t *slot);

/*
 * Enqueue `ticks` time steps of every running member (fewer if all members
 * finish).  A member that takes its last step also gets its final work
 * (last trace row, or the extraction p_adj = tau'^T v_0) and completes.
 * Each call records an event that el_group_sync waits for.
 */
el_status el_group_run(el_group g, int32_t ticks);

/* Block until at most `pending` of the el_group_run calls so far are still
 * running on the device; pending = 0: until everything enqueued on the group
 * (runs, joins, withdrawals) has completed.  Bounds how far the host runs
 * ahead of the device, and releases the calls' events. */
el_status el_group_sync(el_group g, int32_t pending);

/* Non-blocking: *steps_done = steps enqueued for the slot's member so far;
 * *done = 1 once its operation (or its withdrawal) has completed on the
 * device, and the slot is then free.  Either pointer may be NULL. */
el_status el_group_poll(el_group g, int32_t slot, int32_t *steps_done, int32_t *done);

/* Withdraw the slot's member: it takes no further steps and its output is
 * left incomplete; the slot frees once the work already enqueued for it has
 * completed (el_group_poll). */
el_status el_group_remove(el_group g, int32_t slot);

/* Number of slots, slots in use, and members still taking steps. */
el_status el_group_members(el_group g, int32_t *total, int32_t *used, int32_t *running);

#ifdef __cplusplus
}
#endif

#endif /* EL_H */
