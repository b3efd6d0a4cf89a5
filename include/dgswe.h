/*
 * dgswe.h - C ABI of the MI355X (gfx950) discontinuous Galerkin shallow
 * water step.
 *
 * The method (arXiv 2508.21208, "GPU-acceleration of the Discontinuous
 * Galerkin Shallow Water Equations Model (DG-SWEM) with OpenACC"):
 *   - 2-D depth-averaged shallow water equations in (zeta, Hu_x, Hu_y) form
 *     with bathymetry h_b positive downward and H = zeta + h_b
 *     (Sec. 2.1, Eq. SWE; Sec. 2.2, Eq. cons_form);
 *   - element weak form with a numerical flux coupling neighbours
 *     (Sec. 2.2, Eq. elem_weak_form): local Lax-Friedrichs, or Roe's flux
 *     on edges wet on both sides (the two fluxes the paper names);
 *   - orthogonal Dubiner modal basis, diagonal mass matrix, p = 1 (the
 *     paper's) or p = 2 (Sec. 2.2, Eq. dubiner);
 *   - explicit SSP Runge-Kutta time stepping of the semi-discrete system
 *     (Sec. 2.2, Eq. RKSSP): SSP-RK(2,2) by default, SSP-RK(3,3) and the
 *     optimal SSP-RK(s,2), s = 3..5; each stage followed by a slope limiter
 *     (face-neighbour or vertex-based) and wetting/drying;
 *   - boundaries: land (no normal flow) and ocean (prescribed tidal
 *     elevation) (Sec. 2.1 boundary partition; Sec. 6.1 tidal forcing);
 *   - sources: bathymetric slope, Manning bottom friction, wind stress and
 *     atmospheric pressure gradient, Coriolis, rain (Sec. 2.1 source list),
 *     the wind and pressure from a moving Holland parametric hurricane or
 *     static nodal fields.
 *
 * Conventions shared by every entry point:
 *   - Element vertices are counter-clockwise; local edge l of an element lies
 *     opposite its vertex l.  The reference triangle has vertices (-1,-1),
 *     (1,-1), (-1,1) mapped to the element's vertices 0, 1, 2.
 *   - State layout w[(var*nm + mode)*n_elems + e] in FP64, var in
 *     {zeta [m], Qx [m^2/s], Qy [m^2/s]}, nm = 3 modes per variable at
 *     p = 1 and 6 at p = 2, in the order of the Dubiner basis (Sec. 2.2)
 *     [phi_00 = 1, phi_10 = A, phi_01 = (1 + 3 eta)/2, phi_20 = (3 A^2 - B^2)/2,
 *     phi_11 = A (3 + 5 eta)/2, phi_02 = (5 eta^2 + 2 eta - 1)/2] with
 *     A = (1 + 2 xi + eta)/2, B = (1 - eta)/2, elements in the caller's order.  The library reorders elements
 *     internally; this is never visible at the boundary.
 *   - Every pointer argument is HOST memory, read only during the call; the
 *     caller keeps ownership and may free it when the call returns.  Output
 *     buffers are allocated by the caller.  All device memory is owned by the
 *     solver and released by dgswe_destroy.
 *   - Every call returns a dgswe_status; nothing throws across the boundary
 *     (a failed host allocation returns DGSWE_E_NOMEM).
 *     On DGSWE_E_INVALID / DGSWE_E_MESH / DGSWE_E_NOMEM the handle (if any)
 *     is left unchanged.  dgswe_last_error gives a message for the last
 *     failed call on a handle.
 *   - One handle per host thread at a time.  Distinct handles on distinct
 *     streams are independent.
 */
#ifndef DGSWE_H
#define DGSWE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgswe_solver dgswe_solver;

typedef enum {
  DGSWE_OK = 0,
  DGSWE_E_INVALID = 1,   /* bad argument or unsupported option */
  DGSWE_E_MESH = 2,      /* mesh fails validation */
  DGSWE_E_NOMEM = 3,     /* device or host allocation failed */
  DGSWE_E_DEVICE = 4,    /* a HIP call failed */
  DGSWE_E_NONFINITE = 5, /* a kernel produced a NaN/Inf */
  DGSWE_E_ALLDRY = 6     /* CFL time step undefined: no wet element and no dt cap */
} dgswe_status;

enum { DGSWE_BC_LAND = 1, DGSWE_BC_OCEAN = 2, DGSWE_BC_RIVER = 3 /* reserved: rejected */ };
enum { DGSWE_FP64 = 0, DGSWE_MIXED = 1 };

typedef struct {
  int32_t p;         /* polynomial degree: 1 or 2 (all members of a batch) */
  int32_t precision; /* DGSWE_FP64, or DGSWE_MIXED (see below) */
  double g;          /* gravity [m/s^2], e.g. 9.81 */
  double rho0;       /* water density [kg/m^3], e.g. 1000 */
  double h0;         /* wet/dry threshold depth H0 [m], e.g. 0.01 */
  double cfl;        /* CFL number, used when dt_fixed <= 0 */
  double dt_fixed;   /* > 0: fixed time step [s] */
  double dt_max;     /* > 0: upper bound on the CFL time step [s] */
  int32_t limiter;   /* slope limiter after each stage: 0 off; 1 face-neighbour
                        (the range of the element's and its face neighbours'
                        means bounds its vertex values); 2 vertex-based, p = 1
                        only (the range of the means of all elements sharing a
                        mesh node bounds the value at that vertex; keeps linear
                        fields on any element whose vertices each lie inside
                        the hull of the surrounding centroids) */
  int32_t wetdry;    /* 1: wetting/drying after each stage */
  int32_t rk;        /* time stepper: 22 = SSPRK(2,2), 33 = SSPRK(3,3),
                        32, 42, 52 = SSPRK(s,2) with s = 3, 4, 5 stages */
  int32_t flux;      /* numerical flux: 0 = local Lax-Friedrichs, 1 = Roe */
  int32_t chunk;     /* launch tuning: elements per workgroup chunk, 64..256
                        (0: chosen per mesh - at p = 1 the largest size up
                        to 256 whose LDS lets the most stage workgroups share
                        a compute unit, else 256); results do not depend on
                        it */
  int32_t waves;     /* launch tuning: waves per SIMD the p = 2 stage kernel's
                        registers are budgeted for, 1..4 (0: 3 in FP64, 2 in
                        mixed precision) */
  int32_t persistent; /* launch tuning: 0 = one workgroup per chunk; N > 0 =
                        N resident workgroups per compute unit, each taking
                        chunks in turn (the same chunks per XCD); results do
                        not depend on it */
} dgswe_params;

/* Numerical flux (Sec. 2.2 names local Lax-Friedrichs and Roe).  flux = 1
 * uses Roe's flux (Roe averages of the velocity with square-root depth
 * weights, c = sqrt(g (H_L + H_R)/2), Harten-Hyman entropy fixes on the
 * acoustic waves) on interior and ocean edges whose two sides are wet; an
 * edge with a dry side keeps the local Lax-Friedrichs wet/dry rules, and a
 * point without positive depth on a side falls back to LLF. */

/* Time steppers (Sec. 2.2: the paper names "optimized" SSP Runge-Kutta
 * schemes without their coefficients).  Every stage is followed by the
 * slope limiter and the wet/dry step; stage k of a step evaluates the
 * forcing and the tide at t^n + c_k dt.
 *   22: SSPRK(2,2), c = (0, 1) (the default).
 *   33: SSPRK(3,3): w1 = w + dt L(w); w2 = 3/4 w + 1/4 (w1 + dt L(w1));
 *       w^{n+1} = 1/3 w + 2/3 (w2 + dt L(w2)); c = (0, 1, 1/2).
 *   s2 (s = 3, 4, 5): SSPRK(s,2): s - 1 Euler steps of dt/(s - 1), then
 *       w^{n+1} = 1/s w + (s - 1)/s (w_{s-1} + dt/(s - 1) L(w_{s-1}));
 *       c_k = k/(s - 1).  Its SSP coefficient is s - 1: the CFL number may
 *       be s - 1 times that of SSPRK(2,2) for the same stability.
 * dt is formed from cfl as for every scheme; choose cfl accordingly. */

/* Precision.  DGSWE_FP64 computes and stores everything in FP64.
 * DGSWE_MIXED (the paper computes in FP32 throughout, Sec. 5) keeps in
 * FP64 the zeta modes, the bathymetry, element areas, every slope-limiter
 * and wet/dry operation, the hydrostatic term and the zeta jump of the
 * flux, the zeta right-hand side and its Runge-Kutta update; the momentum
 * modes are stored in FP32 and the flux, volume and source arithmetic runs
 * in FP32.  Each edge's mass flux is added to one element and subtracted
 * from the other in FP64, so the total mass is conserved to FP64 rounding
 * in both modes.  States cross this interface as FP64 in both modes (the
 * momentum rounded to FP32 on dgswe_set_state).
 *
 * Degree p = 2 (the paper builds p = 1 and states that the formulation
 * extends to higher degrees, Sec. 2.2): six modes per variable, a degree-4
 * six-point area rule and four-point Gauss-Lobatto edges.  The limiter
 * scales modes 1-5 of each variable by the largest factor <= 1 that keeps
 * the field inside the range of the element's and its face neighbours'
 * means at the vertices and edge midpoints (the p = 1 limiter when the
 * quadratic modes vanish); the wet/dry step leaves a dry element (mean
 * depth <= H0) flat and at rest and, in a wet element whose depth falls
 * below H0 at a vertex, an interior edge quadrature point or an area
 * point, scales the depth's deviation from its mean so that the lowest of
 * those points is at H0.  Both are continuous in the state.  The CFL
 * number should be smaller than at p = 1 (about 0.1). */

/* Fill `p` with the defaults: p=1, FP64, g=9.81, rho0=1000, h0=0.01,
 * cfl=0.2, dt_fixed=0, dt_max=0, limiter=1, wetdry=1, rk=22, flux=0, chunk=0,
 * waves=0, persistent=0. */
void dgswe_default_params(dgswe_params *p);

/* Environment variables read when a solver, batch or pool is created (for
 * tuning and testing; none of them changes any result, bitwise):
 *   DGSWE_CHUNK=n          chunk size (64..256, or 0: chosen per mesh),
 *                          overrides params.chunk;
 *   DGSWE_BLOCK=n          stage-kernel block size (only 256 is accepted);
 *   DGSWE_RHS2_WPE=n       p = 2: waves per SIMD the right-hand-side kernel's
 *                          registers are held to (1..4), overrides
 *                          params.waves (read once per process, at the
 *                          first p = 2 step);
 *   DGSWE_FORCING_EVERY_STAGE=1
 *                          evaluate the hurricane forcing at every stage
 *                          instead of reusing the last stage's for the next
 *                          step's first stage (the same time). */

/* Build a solver for one mesh and allocate its device-resident state.
 * (Sec. 2.2: the triangulation Omega = union of elements; Sec. 2.1: the
 * boundary partition into ocean and land sections.)
 *   n_nodes, node_xy [n_nodes][2] (m), node_hb [n_nodes] (bathymetry, m,
 *     positive downward);
 *   n_elems, tri [n_elems][3] (0-based node ids, counter-clockwise);
 *   n_bnd, bnd_nodes [n_bnd][2], bnd_type [n_bnd]: every edge that belongs
 *     to exactly one triangle, typed DGSWE_BC_LAND or DGSWE_BC_OCEAN;
 *   prm: parameters (copied);
 *   hip_stream: a hipStream_t to enqueue all work on, or NULL for a stream
 *     owned by the solver;
 *   out: receives the handle (NULL on error).
 * Validation: indices in range, positive (counter-clockwise) area, no edge
 * shared by more than two triangles, every boundary edge typed exactly
 * once -> otherwise DGSWE_E_MESH; DGSWE_BC_RIVER, p not 1 or 2, or an
 * unsupported precision -> DGSWE_E_INVALID.  The initial state is zero at t = 0. */
dgswe_status dgswe_create_mesh(int32_t n_nodes, const double *node_xy, const double *node_hb,
                               int32_t n_elems, const int32_t *tri, int32_t n_bnd,
                               const int32_t *bnd_nodes, const int32_t *bnd_type,
                               const dgswe_params *prm, void *hip_stream, dgswe_solver **out);

/* One mesh of a batch: the arguments of dgswe_create_mesh. */
typedef struct {
  int32_t n_nodes;
  const double *node_xy;
  const double *node_hb;
  int32_t n_elems;
  const int32_t *tri;
  int32_t n_bnd;
  const int32_t *bnd_nodes;
  const int32_t *bnd_type;
} dgswe_mesh;

/* A batch: n_meshes independent instances of the same step (an ensemble of
 * storm tracks, a queue of requests), advanced together by dgswe_step with
 * one kernel launch per stage for all of them.  The paper runs one mesh;
 * a member of a batch follows exactly the same arithmetic as that mesh
 * alone (same results, bitwise), with its own forcing, time, dt (its own
 * CFL minimum), step count and error status.  Parameters (prm, including
 * the precision) are shared.  Each mesh is validated as in
 * dgswe_create_mesh (errors name the mesh); at most 2^31 - 1 elements in
 * total.  A handle made by dgswe_create_mesh is a batch of one.  The
 * single-mesh calls (dgswe_set_state, dgswe_set_forcing, dgswe_read_state)
 * return DGSWE_E_INVALID on a batch of several meshes; use the member calls
 * below, whose `member` is the index into `meshes` (out of range ->
 * DGSWE_E_INVALID). */
dgswe_status dgswe_create_batch(int32_t n_meshes, const dgswe_mesh *meshes, const dgswe_params *prm,
                                void *hip_stream, dgswe_solver **out);

/* Number of member slots (meshes of a batch, capacity of a pool; 0 for
 * NULL). */
int32_t dgswe_member_count(const dgswe_solver *s);

/* A serving pool: an empty batch whose members join and leave between
 * dgswe_step calls (continuous batching, as in a serving loop).  The
 * device memory is reserved here once: room for max_elems elements in total
 * (with the matching node, halo and edge storage) and max_members member
 * slots.  A joining mesh takes a contiguous range of each store (first
 * fit); a leaving one gives it back.  Every step advances all members
 * present, each with its own forcing, time, dt and status, with one kernel
 * launch per stage over exactly the present members' work; a member's
 * results do not depend on what else is in the pool (bitwise).  Members
 * are addressed by slot (the member calls above).  Capacity out of range
 * (max_elems in [1, 2^30 - 1], max_members in [1, 65536]) or invalid
 * params -> DGSWE_E_INVALID; device memory exhausted -> DGSWE_E_NOMEM. */
dgswe_status dgswe_create_pool(int64_t max_elems, int32_t max_members, const dgswe_params *prm, void *hip_stream,
                               dgswe_solver **out);

/* A mesh after host-only preprocessing (validation, element ordering, halo
 * and edge tables) for the order and precision of `prm`: thread safe, no
 * device work, so a serving loop can prepare arriving requests while the
 * device steps.  Errors as dgswe_create_mesh. */
typedef struct dgswe_prepared dgswe_prepared;
dgswe_status dgswe_prepare_mesh(const dgswe_mesh *mesh, const dgswe_params *prm, dgswe_prepared **out);
void dgswe_prepared_free(dgswe_prepared *p);
int64_t dgswe_prepared_elems(const dgswe_prepared *p);

/* Admit a prepared mesh into a free slot of a pool (state zero at t = 0, no
 * forcing; then dgswe_member_set_forcing / dgswe_member_set_state).  On
 * success the pool owns `p` (do not free it) and *member receives the slot.
 * On any error the pool is unchanged and the caller keeps `p` (free it or
 * try again later).  Admission is by memory: no free slot or no contiguous
 * room in some store -> DGSWE_E_NOMEM; `p` prepared for another order p,
 * or `s` not a pool -> DGSWE_E_INVALID.
 * Waits for the stream (the step tables are rewritten). */
dgswe_status dgswe_member_add_prepared(dgswe_solver *s, dgswe_prepared *p, int32_t *member);

/* dgswe_prepare_mesh + dgswe_member_add_prepared in one call. */
dgswe_status dgswe_member_add(dgswe_solver *s, const dgswe_mesh *mesh, int32_t *member);

/* Release a member's slot and storage (waits for the stream; read its state
 * first).  Empty slot or not a pool -> DGSWE_E_INVALID. */
dgswe_status dgswe_member_remove(dgswe_solver *s, int32_t member);

/* Pool occupancy: out[0] elements in use, out[1] element capacity,
 * out[2] members present, out[3] slots, out[4] device bytes held. */
dgswe_status dgswe_pool_usage(const dgswe_solver *s, int64_t out[5]);

/* Replace the modal state (layout above, caller's element order) and set the
 * time to t; resets the step counter.  `w` is copied before the call returns.
 * Every stage of the step starts from a post-processed state (slope limiter,
 * then wet/dry: a wet element has depth >= h0 at its vertices, a dry one is
 * flat and at rest).  postprocess != 0 applies that post-processing once to
 * `w` (use it for initial conditions); 0 takes `w` as is (use it to resume
 * from a state returned by dgswe_read_state: the continuation is then
 * bitwise identical to an uninterrupted run). */
dgswe_status dgswe_set_state(dgswe_solver *s, double t, const double *w, int32_t postprocess);

/* dgswe_set_state for one member of a batch (w: that mesh's elements).
 * The other members are not touched; the member's time, dt and step count
 * restart from t. */
dgswe_status dgswe_member_set_state(dgswe_solver *s, int32_t member, double t, const double *w,
                                    int32_t postprocess);

/* Forcing (Sec. 2.1: bottom friction tau_b, sources F_x, F_y; Sec. 6.1:
 * tidal elevation on the open boundary).
 *   manning_n: Manning coefficient, or per element via manning_n_elem
 *     [n_elems] (caller's order) when non-NULL; friction
 *     -g n^2 |Q| Q / max(H, h0)^(7/3);
 *   tide: zeta_b(t) = tide_offset + sum_i amp_i cos(omega_i t + phase_i),
 *     n_tide <= 8, imposed on ocean edges with the interior momentum;
 *   wind_tau [n_nodes][2] (N/m^2) and patm [n_nodes] (Pa): static nodal
 *     fields (either may be NULL), used when holland == 0;
 *   holland != 0: Holland (1980) vortex centred at (x0 + vx t, y0 + vy t),
 *     central pressure pn - dp, radius of maximum wind rmax, shape B, air
 *     density rho_air, Coriolis parameter coriolis_f, surface wind =
 *     wind_factor x gradient wind, stress rho_air Cd |W| W with
 *     Cd = min(3.5e-3, (0.75 + 0.067 |W|) 1e-3), evaluated at the nodes at
 *     every stage time. */
typedef struct {
  double manning_n;
  const double *manning_n_elem;
  int32_t n_tide;
  const double *tide_amp, *tide_omega, *tide_phase;
  double tide_offset;
  const double *wind_tau;
  const double *patm;
  int32_t holland;
  double x0, y0, vx, vy, dp, pn, rmax, B, rho_air, coriolis_f, wind_factor;
  double coriolis;   /* Coriolis parameter f of the momentum equations (1/s):
                        S_Qx += f Qy, S_Qy -= f Qx in wet elements; 0: off */
  double rain;       /* uniform rainfall rate R (m/s): S_zeta += R everywhere
                        (Sec. 2.1 lists both among the sources) */
} dgswe_forcing;

dgswe_status dgswe_set_forcing(dgswe_solver *s, const dgswe_forcing *f);

/* dgswe_set_forcing for one member of a batch (arrays sized for its mesh). */
dgswe_status dgswe_member_set_forcing(dgswe_solver *s, int32_t member, const dgswe_forcing *f);

/* Enqueue n_steps time steps of every member, with the SSP Runge-Kutta
 * scheme params.rk selects (SSPRK(2,2) by default; the list is above), on
 * the solver's stream and return without waiting (Sec. 2.2, Eq. RKSSP;
 * Sec. 5.2, Algorithms 1-3).  Each step computes its dt on the device, per member: dt_fixed if
 * > 0, otherwise cfl * min over the member's wet elements of
 * 2 r_e / (|Q_mean|/H_mean + sqrt(g H_mean)) (r_e the inradius), capped by
 * dt_max if > 0.  Errors detected by the kernels (DGSWE_E_NONFINITE,
 * DGSWE_E_ALLDRY) stop all further steps of that member and are reported
 * by its next read. */
dgswe_status dgswe_step(dgswe_solver *s, int32_t n_steps);

/* Advance a p = 1 solver (batch or pool) and a p = 2 solver together by
 * n_steps steps, for ensembles whose members have both orders (Sec. 2.2:
 * the formulation carries to higher degrees).  Per RK stage one launch
 * does the stage of every p = 1 chunk together with the post-processing
 * (limiter, wet/dry) of every p = 2 chunk, then one launch the p = 2
 * right-hand side (the environment variable DGSWE_PAIR_SPLIT=0 selects the
 * other arrangement: the p = 2 post-processing, then one launch of both
 * orders' stage work); each member's result is bitwise the one dgswe_step
 * gives its solver alone.  The two must share
 * the device, the precision, the time stepper and the persistent setting,
 * and p1 must not use the vertex-based limiter (DGSWE_E_INVALID otherwise).
 * The work runs on p1's stream; if p2 has another stream, p2's earlier work
 * is waited for and p2's later work waits for the pair.  p1's
 * steps_per_graph (dgswe_use_graphs) applies to the pair.  Asynchronous
 * like dgswe_step; errors are reported by each solver's next read. */
dgswe_status dgswe_step_pair(dgswe_solver *p1, dgswe_solver *p2, int32_t n_steps);

/* Step graphs: steps_per_graph > 0 (rounded up to a multiple of 6) makes
 * dgswe_step enqueue its steps in whole graphs of that many steps, each
 * captured once (per buffer rotation and step parity) into a HIP graph and
 * replayed, and the remainder launch by launch; 0 turns graphs off.  The
 * results are bitwise those of the launches themselves.  Graphs are dropped
 * and recaptured when the launch tables change (members join or leave,
 * forcing changes); profiling (dgswe_profile) uses the plain launches.  For
 * small meshes, where a stage takes a few microseconds, this removes the
 * per-launch host cost. */
dgswe_status dgswe_use_graphs(dgswe_solver *s, int32_t steps_per_graph);

typedef struct {
  double t;        /* model time [s] */
  double dt_last;  /* dt of the last step [s] */
  double mass;     /* sum_e A_e zeta_mean_e [m^3] */
  double volume;   /* sum_e A_e H_mean_e [m^3] */
  int64_t steps;   /* steps since dgswe_set_state */
  int32_t n_wet, n_dry;
} dgswe_diag;

/* Wait for the solver's stream, then copy the state (if w_out != NULL, same
 * layout as dgswe_set_state) and the diagnostics (if d != NULL).  Returns
 * the first kernel-detected error, if any (the data are still copied). */
dgswe_status dgswe_read_state(dgswe_solver *s, double *w_out, dgswe_diag *d);

/* dgswe_read_state for one member of a batch (its own diagnostics and
 * error status). */
dgswe_status dgswe_member_read_state(dgswe_solver *s, int32_t member, double *w_out, dgswe_diag *d);

/* For callers that cannot allocate memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The read-back of
 * dgswe_member_read_state without allocating, copying to the host or
 * waiting: it enqueues on the solver's stream
 *   - the member's post-processed state into w_dev (if not NULL): device
 *     memory owned by the caller, FP64 [3][nmodes][n_elems] in the caller's
 *     element order, exactly what dgswe_member_read_state writes;
 *   - its diagnostics into diag_dev (if not NULL): device memory of 8
 *     doubles, t, dt_last, mass, volume, steps, n_wet, n_dry and the
 *     member's device status word (0, or the DGSWE_E_* a kernel reported);
 * and returns.  The values are in place once the stream has run that far.
 * Scratch: the diagnostics' partial sums live in one static device array
 * per GPU (1.5 MiB, held until the process ends) sized for members of at
 * most DGSWE_NOALLOC_MAX_ELEMS elements; a larger member gives
 * DGSWE_E_INVALID and enqueues nothing.  Every call on a GPU uses that
 * GPU's array: calls on one GPU that overlap (different streams with no
 * ordering between them) race and may mix their diagnostics. */
#define DGSWE_NOALLOC_MAX_ELEMS 16777216
dgswe_status dgswe_member_read_state_device(dgswe_solver *s, int32_t member, double *w_dev, double *diag_dev);

/* Release the solver and its device memory (NULL is ignored). */
void dgswe_destroy(dgswe_solver *s);

/* Message for the last failed call on `s` (or the last failed
 * dgswe_create_mesh in this thread when s is NULL).  Never NULL. */
const char *dgswe_last_error(const dgswe_solver *s);

/* Kernel timing with HIP events on the solver's stream.  enable != 0 starts
 * recording (and clears earlier records); 0 stops. */
dgswe_status dgswe_profile(dgswe_solver *s, int32_t enable);

/* Per-kernel totals since profiling was enabled: for up to max_kernels
 * kernels writes a NUL-terminated name into names + 32*i (32 bytes each),
 * the summed duration in ms and the launch count.  *n_out receives the
 * number of kernels written.  Waits for the stream. */
dgswe_status dgswe_profile_read(dgswe_solver *s, int32_t max_kernels, char *names, double *total_ms,
                                int64_t *launches, int32_t *n_out);

/* Sizes after preprocessing: out[0] = nodes, out[1] = elements,
 * out[2] = edges, out[3] = boundary edges (the sums over a batch). */
dgswe_status dgswe_mesh_info(const dgswe_solver *s, int64_t out[4]);

/* The same sizes for one member of a batch. */
dgswe_status dgswe_member_info(const dgswe_solver *s, int32_t member, int64_t out[4]);

#ifdef __cplusplus
}
#endif

#endif /* DGSWE_H */
