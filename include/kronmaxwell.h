/*
 * kronmaxwell - explicit leapfrog of the spline geometric Maxwell scheme with
 * Kronecker-structured pairing solves (Kapidani & Vazquez, "High order
 * geometric methods with splines: fast solution with explicit time-stepping
 * for Maxwell equations"), for AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2-3 of the paper): Maxwell's equations in differential forms
 * on the unit cube mapped by F, with perfect-conductor walls,
 *     d_t D = dH - J,   d_t B = -dE,   D = eps E (via a Hodge star), B = mu H.
 * E and B live in the primal spline complex of degrees p / p-1 with boundary
 * conditions built in (X^1_{h,0}, X^2_{h,0}); H and D in the dual complex of
 * degrees p-1 / p-2 (X~^1, X~^2).  The scheme of Section 3.4, eqs. (3.10)-(3.13),
 * uses the Hodge operators of the second kind:
 *     K1 e = M~^2_{1/eps} d,      K~1 h = M^2_{1/mu} b,
 * so every time step applies the geometry/material mass matrices M and solves
 * with the metric-free pairing matrices K1, K~1, whose blocks are Kronecker
 * products of 1D matrices (eqs. (4.2)-(4.5)).
 *
 * Discrete unknowns and their layout in device memory (all FP64):
 *   e  (X^1_{h,0}) and d (X~^2): n_e = 3 * n1 * n0^2 values
 *   h  (X~^1)      and b (X^2_{h,0}): n_h = 3 * n0 * n1^2 values
 * with n0 = N + p - 2, n1 = N + p - 1 for N elements per axis.  A vector stores
 * its three components one after the other; inside a component the x index
 * runs fastest.  Component c of e has n1 entries along axis c and n0 across,
 * component c of h has n0 along axis c and n1 across.
 *
 * Time stepping (staggered leapfrog, Petrov-Galerkin (e, h) form of Section
 * 3.4.2 with the tested source s = M~ j):
 *     h^{n+1/2} = h^{n-1/2} - dt K~1^{-1} M^2_{1/mu} D^1 e^n
 *     e^{n+1}   = e^n + dt K1^{-1} ( M~^2_{1/eps} D~^1 h^{n+1/2} - s(t_{n+1/2}) )
 * and, when tracking is on, b^{n+1/2} = b^{n-1/2} - dt D^1 e^n and
 * d^{n+1} = d^n + dt D~^1 h^{n+1/2}.
 *
 * Conventions for every call:
 *   - Each call returns a kmx_status; nothing throws across this interface;
 *     kmx_last_error() gives a thread-local message for the last failure.
 *   - Pointers documented as "device" are HIP device pointers owned by the
 *     caller; pointers documented as "host" are ordinary host memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Device work is
 *     enqueued on it; calls that return host results synchronise it.
 *   - The space owns all operator data and all scratch memory, sized at
 *     creation for `max_batch` fields; kmx_step never allocates.
 *   - Calls on one space must not overlap on different streams (they share
 *     the space's scratch memory).
 */
#ifndef KRONMAXWELL_H
#define KRONMAXWELL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kmx_space kmx_space;
typedef struct kmx_source kmx_source;
typedef struct kmx_probes kmx_probes;
typedef struct kmx_graph kmx_graph;

typedef enum {
    KMX_OK = 0,
    KMX_E_ARG = 1,       /* invalid argument (size, pointer, degree, batch) */
    KMX_E_GEOMETRY = 2,  /* det DF <= 0 (or not finite) at a quadrature point */
    KMX_E_MATERIAL = 3,  /* eps or mu <= 0 or not finite */
    KMX_E_DEVICE = 4,    /* a HIP runtime call failed */
    KMX_E_OOM = 5,       /* device allocation failed at creation */
    KMX_E_UNSTABLE = 6,  /* non-finite value detected, or |dt| above the stable step that
                            kmx_cfl (kmx_cfl_scheme1) last computed for the space */
    KMX_E_STATE = 7      /* call not valid in the current state */
} kmx_status;

/* Map of the parametric cube (Section 2.3).
 *   kind 0: identity, Omega = (0,1)^3.
 *   kind 1: x -> x + amplitude * sin(pi x) sin(pi y) sin(pi z) on every
 *           component (a deformed cube, identity on the boundary).
 *   kind 2: user Jacobian: dF_qp (host) holds DF at every quadrature point,
 *           9 doubles row-major (DF[i][j] = dF_i/dx^_j) per point, points in
 *           the order of kmx_quad_points. */
typedef struct {
    int kind;
    double amplitude;
    const double* dF_qp;
} kmx_map;

/* KMX_FP64: every operation in FP64.
 * KMX_MIXED: the pairing solves x = K^{-1} y of the time step (eqs.
 * (4.4)-(4.5)) use dense inverses of the 1D factors, rounded to FP32 and
 * applied as mode-n products on the matrix cores with FP32 accumulation; the
 * result is corrected by iterative refinement x += K^{-1}_32 (y - K x) whose
 * residual uses the FP64 banded factors (kmx_set_refinement sets the number of
 * corrections, default 2).  Hodge applies, curls, updates, the 1D
 * factorisations and the energy sums stay FP64.  Mixed spaces always run the
 * tiled plan. */
typedef enum { KMX_FP64 = 0, KMX_MIXED = 1 } kmx_precision;

/* OR into the `precision` argument of kmx_create_space to stream the metric
 * factor w_q DF^T DF / det DF from device memory (6 doubles per quadrature
 * point) even for map kinds 0 and 1, whose factor is otherwise recomputed at
 * every quadrature point inside the mass kernel.  Map kind 2 always streams. */
#define KMX_STORED_METRIC 16

/* Number of FP64-residual corrections of a mixed-precision solve (0..8). */
kmx_status kmx_set_refinement(kmx_space* sp, int steps);

/* flags for kmx_step / kmx_init_stagger */
#define KMX_TRACK_DB 1 /* E holds [e | d] and H holds [h | b] per batch member */

/* Create the discrete spaces, operators and scratch for degree p (2..4),
 * n_elem elements per axis (1..72), map `map` (host struct), precision, and at
 * most max_batch simultaneous fields.  Materials default to eps = mu = 1.
 * Uses the current HIP device.  Gauss rule: p+1 points per element and axis.
 * Errors: KMX_E_ARG, KMX_E_GEOMETRY, KMX_E_OOM, KMX_E_DEVICE. */
kmx_status kmx_create_space(int p, int n_elem, const kmx_map* map, int precision,
                            int max_batch, kmx_space** out);

/* Release everything the space owns (NULL is accepted). */
void kmx_destroy_space(kmx_space* sp);

/* Per-element eps and mu (host, N^3 each, element index x fastest); NULL keeps
 * the value 1.  Forgets the stable steps computed by kmx_cfl and
 * kmx_cfl_scheme1 (they depend on the materials).  Errors: KMX_E_MATERIAL,
 * KMX_E_DEVICE; KMX_E_STATE while graphs captured on the space exist (a
 * graph holds the material state it was captured with: destroy it first). */
kmx_status kmx_set_materials(kmx_space* sp, const double* eps_elem, const double* mu_elem);

/* n_e = dim X^1_{h,0} = dim X~^2, n_h = dim X~^1 = dim X^2_{h,0}, n_qp = number
 * of quadrature points (N^3 (p+1)^3).  Any output pointer may be NULL. */
kmx_status kmx_sizes(const kmx_space* sp, int64_t* n_e, int64_t* n_h, int64_t* n_qp);

/* Physical coordinates F(x^_q) of every quadrature point, host array of
 * 3 * n_qp doubles, element-major: [ez][ey][ex][iqz][iqy][iqx][xyz].  For map
 * kind 2 only the Jacobians are known: the parametric coordinates x^_q are
 * returned (the caller maps them). */
kmx_status kmx_quad_points(const kmx_space* sp, double* xyz_host);

/* Initial electric field (Section 5.1, "projecting" the initial data):
 * e = K1^{-1} l with l_i = int_Omega eta_i . E0 dx over the dual 2-form basis
 * eta_i, the L^2_{1/eps} projection of D0 = eps E0 followed by the Hodge (3.11).
 * E_qp_host: physical E0 at the quadrature points (3 * n_qp doubles, order of
 * kmx_quad_points).  e_dev: device, n_e doubles (written).  Host computation
 * plus one copy on `stream`. */
kmx_status kmx_project_E(kmx_space* sp, const double* E_qp_host, double* e_dev, void* stream);

/* d = M~^{-1} l (the L^2_{1/eps} projection of D0 itself, for tracking d),
 * by preconditioned conjugate gradients on the device to relative residual
 * `tol`.  E_qp_host as for kmx_project_E; d_dev: device, n_e doubles. */
kmx_status kmx_project_D(kmx_space* sp, const double* E_qp_host, double* d_dev, double tol,
                         void* stream);

/* Largest stable step 2 / sqrt(lambda_max(K1^{-1} M~ D~^1 K~1^{-1} M D^1)) by
 * power iteration on the device (seeded start vector), stopping when the
 * eigenvalue estimate changes by less than tol (relative) or after max_iter
 * iterations.  Synchronises.  The space keeps the result: until the next
 * kmx_set_materials, kmx_step and kmx_graph_create refuse |dt| above it, and
 * kmx_step_split a largest substep max_j |c_j dt| above it, with
 * KMX_E_UNSTABLE (before any device work).  Without a kmx_cfl call no step is
 * checked. */
kmx_status kmx_cfl(kmx_space* sp, int max_iter, double tol, double* dt_max);

/* Point dipoles J = q delta(x - F(x^0)) g(t), g(t) = amp exp(-(t - t0)^2 / (2 sigma^2)).
 * Tested source s_i = q . eta_i(x0) / eps(x0) with eta_i the physical dual
 * 2-form basis (pushed forward).  Host arrays: pos (n x 3, parametric position
 * in [0,1]^3), moment (n x 3), t0, sigma, amp (n each), batch_of (n, the batch
 * member each dipole drives; NULL = member 0).  The source keeps a reference
 * to nothing on the host; materials must be set before creating sources. */
kmx_status kmx_create_source(kmx_space* sp, int n, const double* pos, const double* moment,
                             const double* t0, const double* sigma, const double* amp,
                             const int* batch_of, kmx_source** out);
void kmx_destroy_source(kmx_source* src);

/* The other source form: s(t) = g(t) P, a dense time-independent pattern P
 * in the dual 2-form space X~^2 (the tested source vector itself, n_e entries
 * in the layout of d) times a sampled time series g.  pattern (host): npat x
 * n_e doubles, npat = 1 (every batch member) or one pattern per member
 * (steps then need batch <= npat).  series (host): nsamples >= 2 values at
 * t0 + k dt_sample; g(t) is their linear interpolation, zero outside
 * [t0, t0 + (nsamples - 1) dt_sample].  The step subtracts s(t_{n+1/2}) from
 * M~ D~^1 h before the K1 solve, as for point dipoles (Section 3.4).  The
 * arrays are copied; the source keeps no host reference.  Runs with the
 * tiled plans (a forced separable plan: KMX_E_STATE) and not in kmx_adjoint
 * (KMX_E_STATE); KMX_E_ARG for non-finite data, npat outside 1..max_batch,
 * fewer than two samples or dt_sample <= 0. */
kmx_status kmx_create_source_pattern(kmx_space* sp, int npat, const double* pattern, int nsamples, double t0,
                                     double dt_sample, const double* series, kmx_source** out);

/* Backward half kick from t = 0 data: h <- h + dt/2 K~1^{-1} M D^1 e, and with
 * KMX_TRACK_DB also b <- b + dt/2 D^1 e.  E, H: device, batch members of
 * stride n_e*(1+track) and n_h*(1+track). */
kmx_status kmx_init_stagger(kmx_space* sp, const double* E, double* H, double dt, int batch,
                            int flags, void* stream);

/* nsteps leapfrog steps (formulas above), in place.  On entry E holds e^n (and
 * d^n) and H holds h^{n-1/2} (and b^{n-1/2}) at time t = t_start; on exit the
 * state is advanced by nsteps.  J: NULL or a source of this space (not allowed
 * together with KMX_TRACK_DB).  energy_dev: NULL, or device array of
 * nsteps * batch doubles receiving the leapfrog invariant after every step
 * (requires KMX_TRACK_DB; entry k * batch + m is member m's value after step
 * k + 1, all written by the call's work on the stream), evaluated as
 * 1/2 (d.w_e + b.w_h - dt w_h.D^1 e)
 * with w_e = K1 e and w_h = K~1 h formed once per call (one banded pairing
 * apply each) and then updated with the mass applies of the steps (eqs.
 * (3.11), (3.13) on the increments); it equals kmx_energy's first value to
 * rounding.  Never allocates and never synchronises.
 * KMX_E_UNSTABLE when |dt| exceeds the last kmx_cfl result of the space. */
kmx_status kmx_step(kmx_space* sp, double* E, double* H, const kmx_source* J, double t_start,
                    double dt, int nsteps, int batch, int flags, double* energy_dev, void* stream);

/* ---- execution plans and the autotuner -----------------------------------
 * A space runs kmx_step (and the steps captured by kmx_graph_create) with one
 * of two plans:
 *   KMX_PLAN_TILED      any map and materials: per half step a fused curl +
 *                       sum-factorised mass apply over 4^3-element tiles,
 *                       then the per-axis banded pairing solves (Section 4).
 *   KMX_PLAN_SEPARABLE  identity map with eps and mu the same in every
 *                       element: the Hodge matrices are then Kronecker
 *                       products of 1D Gram matrices like the pairings
 *                       (eqs. (4.2)-(4.3)), so each half step is a curl and
 *                       banded mode products along x, y, z.  One persistent
 *                       workgroup per batch member advances it by all nsteps
 *                       with its component tensors in LDS (lines up to 28,
 *                       components up to the device's LDS per workgroup,
 *                       e.g. p = 3, N <= 25).  No per-step energy output.
 *                       Phases: curl over all entries, one pass per mode
 *                       product, update over all entries.
 *   KMX_PLAN_SEPARABLE_FUSED  the same operators with the curl fused into
 *                       the first (z) pass and the update into the last pass.
 *   KMX_PLAN_TILED_W4   the tiled plan with the mass kernel compiled for four
 *                       resident waves per SIMD (registers capped at 128;
 *                       p <= 3, otherwise as KMX_PLAN_TILED).
 *   KMX_PLAN_TILED_DENSE  the tiled plan with the pairing solves applied
 *                       with the dense inverses of the 1D factors (computed
 *                       once on the host in FP64) on the FP64 matrix cores:
 *                       per z plane B_y X B_x^T, then B_z along z, instead of
 *                       banded substitutions.  Lines of at most 80 entries;
 *                       kmx_set_plan fails with KMX_E_ARG otherwise.
 * KMX_PLAN_AUTO (the default) takes the separable plan when it applies and
 * batch >= 32, the tiled plan otherwise.  `threads` is the separable kernels'
 * workgroup size (64..768, multiple of 64).  Forcing a separable plan on a
 * call it cannot serve fails with KMX_E_STATE.  All plans compute the same
 * operators; results differ by rounding only. */
#define KMX_PLAN_AUTO (-1)
#define KMX_PLAN_TILED 0
#define KMX_PLAN_SEPARABLE 1
#define KMX_PLAN_SEPARABLE_FUSED 2
#define KMX_PLAN_TILED_DENSE 3
#define KMX_PLAN_TILED_W4 4
kmx_status kmx_set_plan(kmx_space* sp, int kind, int threads);
kmx_status kmx_get_plan(const kmx_space* sp, int* kind, int* threads);

/* Times the candidate plans on `batch` members (zero fields of its own, J
 * driving them if not NULL, time step dt) over probe_steps steps each after
 * one warm-up step, and keeps the fastest as the space's plan.  Candidates:
 * 0 tiled; 1 tiled-w4; 2 tiled-dense; 3..5 separable with 384, 512, 768
 * threads; 6..7 separable-fused with 512, 768 threads.  ms_out:
 * NULL or host array of KMX_TUNE_CANDIDATES entries receiving the mean ms per
 * step (-1 where a candidate does not apply).  Allocates two fields of
 * working memory; synchronises. */
#define KMX_TUNE_CANDIDATES 8
kmx_status kmx_tune(kmx_space* sp, int batch, int probe_steps, const kmx_source* J, double dt, double* ms_out,
                    void* stream);

/* ---- graph-captured stepping (one graph launch for a chunk of steps) -----
 * kmx_graph_create captures nsteps leapfrog steps (arguments as kmx_step)
 * into a HIP graph on a stream owned by the space.  The source time of the
 * captured steps is read from the space's device clock, which every replay
 * advances by nsteps*dt, so replaying the graph marches in time; E, H, J and
 * energy_dev are bound at capture and must stay valid.  The graph contains
 * kernel nodes only.  It also holds the material state of the capture (the
 * separable plan bakes uniform eps and mu into its launch), so
 * kmx_set_materials is refused while graphs of the space exist.  A graph may
 * be destroyed after its space.  kmx_set_time / kmx_get_time set and read the clock
 * (synchronising). */
kmx_status kmx_graph_create(kmx_space* sp, double* E, double* H, const kmx_source* J, double dt, int nsteps,
                            int batch, int flags, double* energy_dev, kmx_graph** out);
kmx_status kmx_graph_launch(kmx_graph* g, void* stream);
void kmx_graph_destroy(kmx_graph* g);
kmx_status kmx_set_time(kmx_space* sp, double t, void* stream);
kmx_status kmx_get_time(kmx_space* sp, double* t, void* stream);

/* Energies of tracked states (E = [e|d], H = [h|b], at e^n, d^n, h^{n-1/2},
 * b^{n-1/2}), eq. (3.2):
 *   out_host[2k]   = 1/2 (d.K1 e + b.K~1 h - dt (K~1 h).(D^1 e)), the invariant
 *                    1/2 (d^n.M~ d^n + b^{n-1/2}.M b^{n+1/2}) of the leapfrog,
 *   out_host[2k+1] = 1/2 (e^T K~2 d + h^T K2 b), the paper's energy (3.2),
 * for batch member k.  FP64 deterministic reductions.  Synchronises. */
kmx_status kmx_energy(kmx_space* sp, const double* E, const double* H, double dt, int batch,
                      double* out_host, void* stream);

/* ---- operator-level entry points (one step of the path each) ----------- */

/* y = D^1 x (primal, which = 0: x in X^1_{h,0} -> X^2_{h,0}) or y = D~^1 x
 * (dual, which = 1: X~^1 -> X~^2); device vectors of one field. */
kmx_status kmx_op_curl(kmx_space* sp, int which, const double* x, double* y, void* stream);

/* y = M x for which = 0: M^2_{1/mu} on X^2_{h,0}; which = 1: M~^2_{1/eps} on
 * X~^2.  With `curl` = 1 the input is the 1-form and y = M D x (the fused
 * curl + mass apply of the time step).  Device vectors of one field. */
kmx_status kmx_op_mass(kmx_space* sp, int which, int curl, const double* x, double* y,
                       void* stream);

/* x = K^{-1} y (transpose = 0) or K^{-T} y (transpose = 1) with K = K1
 * (which = 1; y in X~^2 layout, x in X^1_{h,0}) or K~1 (which = 0; y in
 * X^2_{h,0}, x in X~^1), eqs. (4.4)-(4.5).  x and y may alias. */
kmx_status kmx_op_solve(kmx_space* sp, int which, int transpose, const double* y, double* x,
                        void* stream);

/* y = K x with K = K1 (which = 1) or K~1 (which = 0). */
kmx_status kmx_op_pairing(kmx_space* sp, int which, const double* x, double* y, void* stream);

/* ---- higher-order symplectic time stepping -------------------------------
 * Symmetric compositions of the leapfrog (kick-drift-kick) of order 2, 4, 6:
 * step weights c_1..c_m with m = 1, 3, 9, from the triple jump
 * c <- (z1 c, z0 c, z1 c), z1 = 1 / (2 - 2^(1/(2k+1))), z0 = 1 - 2 z1 (Yoshida
 * 1990); the paper names pairing the scheme with higher-order symplectic
 * integrators as future work (Section 6).  The state is (e^n, h^)
 * with h^ = h^n + (c_1 dt / 2) K~1^{-1} M D^1 e^n (for order 2 the leapfrog's
 * h^{n-1/2}); one step runs m substeps
 *     h^ -= a_j dt K~1^{-1} M D^1 e;   e += c_j dt K1^{-1} M~ D~^1 h^
 * with a_1 = c_1 and a_j = (c_{j-1} + c_j) / 2, so order 2 is kmx_step.
 * Tracked b and d (KMX_TRACK_DB) follow the same kicks.  No sources, no
 * energy output; the tiled plans only (KMX_E_STATE for a separable plan;
 * KMX_PLAN_AUTO runs the tiled plan).  The stable step shrinks with the
 * largest |c_j| (1.70 at order 4, 2.30 at order 6). */

/* The staggered start of a composed run: h^ = h^0 + (c_1 dt / 2) K~1^{-1} M D^1 e^0
 * (kmx_init_stagger with c_1 dt).  order: 2, 4 or 6. */
kmx_status kmx_init_split(kmx_space* sp, const double* E, double* H, double dt, int order, int batch,
                          int flags, void* stream);

/* nsteps composed steps of the given order (2, 4, 6) on (E, H) as kmx_step
 * lays them out. */
kmx_status kmx_step_split(kmx_space* sp, double* E, double* H, double dt, int nsteps, int order, int batch,
                          int flags, void* stream);

/* ---- non-homogeneous tangential data for E (Section 3.5) ----------------
 * E_h = E_{h,0} + E_{h,b}: the unknowns e are E_{h,0} in X^1_{h,0}; the lifting
 * E_{h,b} lives in the whole primal 1-form space X^1_h (the boundary functions
 * of the full B-spline basis kept: component c has n1 entries along axis c and
 * n0 + 2 across, x fastest; n_ef = 3 n1 (n0 + 2)^2 entries), carried by its
 * boundary coefficients.  With the lifting the second scheme solves
 * (K1)_0 e_0 = M~ d - (K1)_b e_b, with D^1 from X^1_h to X^2_h and the mass of
 * the Hodge K~1 h = M^2_{1/mu} b taking trial functions in the whole X^2_h. */

/* n_ef, the size of a coefficient vector of X^1_h. */
kmx_status kmx_sizes_full(const kmx_space* sp, int64_t* n_ef);

/* Boundary coefficients of the lifting from tangential data (the projection
 * on the trace space that Section 3.5 asks for; reading: one least-squares
 * fit over the six faces of the parametric cube, in the parametric L^2 norm, so
 * that a coefficient on an edge is fitted to both of its faces; exact when
 * the data is the trace of a field of X^1_h).  Eh_faces (host): the pulled-back
 * field E^ = DF^T (E o F) (three parametric components; the caller knows the
 * map on the boundary) at the Gauss points of the faces x^_a = s, face
 * f = 2 a + s, over the two other axes u < v with u fastest:
 * Eh_faces[((f * Q + i_v) * Q + i_u) * 3 + comp], Q = N (p + 1) points per axis
 * at the positions of kmx_quad_points; only the tangential components are
 * used.  eb_full (host, n_ef): the fitted coefficients, zero at the interior
 * functions.  iters (may be NULL): conjugate-gradient iterations of the fit.
 * Synchronous host computation. */
kmx_status kmx_lift_boundary(kmx_space* sp, const double* Eh_faces, double* eb_full, int* iters);

/* Boundary data E_b(x, t) = sum_j g_j(t) E_b^j(x) with g_j(t) = amp_j
 * cos(omega_j t + phase_j) and E_b^j given by its boundary coefficients
 * (eb_full: host, nterms x n_ef; interior entries ignored), nterms <= 8
 * (0 removes the lifting).  Forms, once and in FP64 on the host,
 * v_h^j = K~1^{-1} M_{0,f} D^1_f e_b^j and v_e^j = (K1)_0^{-1} (K1)_b e_b^j and
 * keeps them on the device; then (for every batch member)
 *   kmx_step:         h -= dt g_j(t_n) v_h^j after the h update and
 *                     e -= (g_j(t_{n+1}) - g_j(t_n)) v_e^j after the e update,
 *                     t_n the time at the start of the step (graph replays:
 *                     the space's device clock);
 *   kmx_init_stagger: h += dt/2 g_j(0) v_h^j;
 *   kmx_project_E:    e = K1^{-1} l - g_j(0) v_e^j (the Hodge with the lifting
 *                     at t = 0).
 * The lifting depends on mu, so kmx_set_materials removes it.  Not with
 * KMX_TRACK_DB (KMX_E_ARG), composed steps, the first scheme, the adjoint or
 * a forced separable plan (KMX_E_STATE); KMX_E_STATE while graphs of the space
 * exist.  Allocates its two device arrays (nterms fields each). */
kmx_status kmx_set_lifting(kmx_space* sp, int nterms, const double* eb_full, const double* amp,
                           const double* omega, const double* phase);

/* ---- the first scheme: Hodge stars with 1-form mass matrices -------------
 * Section 3.3, eqs. (3.5)-(3.8): M^1_eps e = K~2 d and M~^1_mu h = K2 b, with
 * K~2 = K1^T and K2 = K~1^T (the pairing-transpose property of Section 2.4),
 * advanced in the (e, h) form of Section 3.3.2 by the same leapfrog:
 *     h^{n+1/2} = h^{n-1/2} - dt (M~^1_mu)^{-1} K~1^T D^1 e^n
 *     e^{n+1}   = e^n + dt (M^1_eps)^{-1} K1^T D~^1 h^{n+1/2}
 * (source free).  M^1_eps (on X^1_{h,0}, n_e unknowns) and M~^1_mu (on X~^1,
 * n_h unknowns) have entries int eta^_i . G1 eta^_j gamma over the parametric
 * cube, G1 = det DF (DF^T DF)^{-1} the covariant pullback factor, gamma = eps or
 * mu per element.  Their systems are solved by conjugate gradients stopped at
 * |y - M x| <= tol |y|, preconditioned with a Kronecker-product approximation
 * of the mass: per component, 1D Gram matrices weighted by the best separable
 * (log-additive) fit of gamma (G1)_cc, inverted exactly.  It is the mass
 * matrix itself when the map is the identity or another orthogonal product
 * map (such as the quarter annulus) and the material is uniform.
 * These calls need an FP64 space (KMX_E_STATE for KMX_MIXED) and allocate, at
 * their first use, eps and mu on the tiles, eight field-sized work vectors
 * and (streamed-metric spaces) the 1-form metric factor; they synchronise the
 * stream while solving (the residual norm is read back) and are not
 * graph-capturable.  One field per call (no batch). */

/* y = M^1_eps x (which = 0, X^1_{h,0}) or y = M~^1_mu x (which = 1, X~^1);
 * device vectors of one field. */
kmx_status kmx_op_mass1(kmx_space* sp, int which, const double* x, double* y, void* stream);

/* x = M^{-1} y for the mass of kmx_op_mass1 (which as there), starting from
 * the guess held in x (device, overwritten; must not alias y).  iters (host,
 * may be NULL) receives the CG iterations.  KMX_E_UNSTABLE when the tolerance
 * is not reached within max_iter iterations or a value is not finite. */
kmx_status kmx_solve_mass1(kmx_space* sp, int which, const double* y, double* x, double tol, int max_iter,
                           int* iters, void* stream);

/* One half step of the first scheme:
 *   which = 1: out += alpha (M~^1_mu)^{-1} K~1^T D^1 x   (x = e, out = h)
 *   which = 0: out += alpha (M^1_eps)^{-1} K1^T D~^1 x   (x = h, out = e)
 * The solve starts from the space's previous solution of the same kind (a
 * warm start).  With which = 1 and alpha = dt/2 it gives the staggered start
 * h^{-1/2} = h^0 + dt/2 (M~^1_mu)^{-1} K~1^T D^1 e^0.  iters as above. */
kmx_status kmx_half_step_scheme1(kmx_space* sp, int which, const double* x, double* out, double alpha, double tol,
                                 int max_iter, int* iters, void* stream);

/* Initial value of the first scheme: e^0 (device, n_e) = the L^2_eps projection
 * of a physical field E0 onto X^1_{h,0}, M^1_eps e^0 = l with
 * l_i = int eps E0 . eta_i dx (eta_i = DF^{-T} eta^_i the primal 1-form basis),
 * solved by the same PCG to tol.  E_qp_host as for kmx_project_E (3 doubles per
 * quadrature point, in the order of kmx_quad_points).  Synchronises. */
kmx_status kmx_project_E1(kmx_space* sp, const double* E_qp_host, double* e_dev, double tol, void* stream);

/* nsteps leapfrog steps of the first scheme on (e^n, h^{n-1/2}) (device, n_e
 * and n_h values).  iters (host, 2 ints, may be NULL) receives the summed CG
 * iterations of the e solves and of the h solves.  KMX_E_UNSTABLE when |dt|
 * exceeds the last kmx_cfl_scheme1 result (also for
 * kmx_graph_create_scheme1). */
kmx_status kmx_step_scheme1(kmx_space* sp, double* e, double* h, double dt, int nsteps, double tol, int max_iter,
                            int* iters, void* stream);

/* nsteps steps of the first scheme on the device arrays e, h captured once as
 * a HIP graph (replayed with kmx_graph_launch, released with
 * kmx_graph_destroy): every mass solve runs a fixed number of preconditioned CG
 * iterations (iters_e, iters_h >= 1; choose them from the counts a tolerance-
 * driven kmx_step_scheme1 reports) with no read-back of the residual, from the
 * warm start of the previous solve.  The space's first-scheme set-up (its
 * allocations) is done before the capture.  The captured graph holds kernel
 * and device-to-device copy nodes only. */
kmx_status kmx_graph_create_scheme1(kmx_space* sp, double* e, double* h, double dt, int nsteps, int iters_e,
                                    int iters_h, kmx_graph** out);

/* Largest stable time step of the first scheme, 2 / sqrt(lambda_max) of
 * (M^1_eps)^{-1} K1^T D~^1 (M~^1_mu)^{-1} K~1^T D^1 by power iteration from the
 * same seeded start as kmx_cfl (stops when lambda changes by at most tol
 * relative), each mass solve to cg_tol.  Allocates two fields; synchronises.
 * The space keeps the result for the checks of kmx_step_scheme1. */
kmx_status kmx_cfl_scheme1(kmx_space* sp, int max_iter, double tol, double cg_tol, double* dt_max);

/* ---- probes and the adjoint (gradient of a probe misfit in eps) ----------
 * Not part of the paper, which has no inverse problem: the exact discrete
 * adjoint of the leapfrog above. */

/* Point probes of the physical electric field E_h(x) = DF^{-T} E^_h(x^) at n
 * parametric positions (host, n x 3, in [0,1]^3).  The probe operator P
 * (3n rows: probe, component) is precomputed on the host and kept on the
 * device.  For map kind 2 the Jacobian of the probe's element's first
 * quadrature point is used. */
kmx_status kmx_create_probes(kmx_space* sp, int n, const double* pos, kmx_probes** out);
void kmx_destroy_probes(kmx_probes* pr);

/* out (device, 3n) = P e for e (device, n_e). */
kmx_status kmx_probe_eval(kmx_space* sp, const kmx_probes* pr, const double* e, double* out, void* stream);

/* From zero fields, nsteps leapfrog steps driven by J (may be NULL); obs
 * (device, nsteps x 3n) receives P e^n for n = 1..nsteps.  Allocates two
 * fields of working memory; synchronises.  Runs the tiled plan, like
 * kmx_adjoint (a separable plan set on the space is restored afterwards). */
kmx_status kmx_probe_forward(kmx_space* sp, const kmx_probes* pr, const kmx_source* J, double dt, int nsteps,
                             double* obs, void* stream);

/* kmx_probe_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same steps and probe values, with the two working fields
 * held in a fixed device array of the library (KMX_NOALLOC_FIELD_MAX doubles
 * per field, 32 MiB per GPU, held until the process ends) instead of memory
 * allocated per call.  Allocates nothing and does not synchronise (stream
 * ordered; errors of the launches are reported, those of the kernels at the
 * caller's next synchronisation).  KMX_E_ARG when n_e or n_h exceeds
 * KMX_NOALLOC_FIELD_MAX.  All calls on one GPU share that array: calls that
 * overlap on one GPU (e.g. on two streams) race. */
#define KMX_NOALLOC_FIELD_MAX (1 << 21)
kmx_status kmx_probe_forward_noalloc(kmx_space* sp, const kmx_probes* pr, const kmx_source* J, double dt,
                                     int nsteps, double* obs, void* stream);

/* Loss L = 1/2 sum_n |P e^n - data_n|^2 over the run of kmx_probe_forward and
 * its gradient with respect to the per-element eps of the space (the eps set
 * by kmx_set_materials; create J after setting them: the tested dipole carries
 * 1/eps at its element), by the discrete adjoint of the leapfrog:
 *   lam = K1^{-T} ebar; hbar += dt D~^{1T} M~ lam;
 *   g_e += -dt/eps_e^2 sum_{q in e} Lam . G (D~^1 h^{n+1/2}) (+ dt g(t) lam.s / eps at the dipole element);
 *   ebar -= dt D^{1T} M K~1^{-T} hbar; ebar += P^T (P e^n - data_n).
 * The forward states are recomputed from checkpoints taken every
 * `checkpoint_every` steps.  data: device, nsteps x 3n.  loss_host: host
 * scalar.  grad: device, N^3 (x fastest), overwritten.  Allocates its working
 * memory (checkpoints, one segment of h, probe values); synchronises.  The
 * forward steps run the tiled plan (the operators the reverse sweep
 * transposes; a separable plan set on the space is restored afterwards).  A
 * failing forward step (e.g. KMX_E_UNSTABLE) ends the call with its status;
 * loss_host and grad are then not valid. */
kmx_status kmx_adjoint(kmx_space* sp, const kmx_probes* pr, const kmx_source* J, const double* data, double dt,
                       int nsteps, int checkpoint_every, double* loss_host, double* grad, void* stream);

/* ---- per-kernel timing ---------------------------------------------------
 * Between kmx_profile_begin and kmx_profile_end every kernel the space
 * launches (up to `capacity` launches) is bracketed by HIP events recorded on
 * the launch stream.  kmx_profile_end waits for the last event and returns,
 * per kernel kind, the summed elapsed milliseconds and the launch count:
 *   0 mass apply on X^2_{h,0} (with the primal curl fused)
 *   1 mass apply on X~^2 (with the dual curl fused)
 *   2 pairing solves (or applies) along x and y
 *   3 pairing solve along z + leapfrog update
 *   4 curl (tracking of b and d)
 *   5 energy reductions
 *   6 patch gather (sum of the overlapping tile outputs of a mass apply)
 *   7 separable persistent kernel (one launch for all steps of a call)
 *   8 FP32 dense mode products of the mixed-precision solves
 *   9 FP64 dense solves of the tiled-dense plan (plane pass and z pass, one
 *     span per solve), and the dense Kronecker applies of the first scheme
 *  10 mass apply on a 1-form space (first scheme)
 *  11 vector updates and dot products of the first scheme's CG
 * Arrays ms_total and launches (host) hold KMX_PROFILE_KINDS entries. */
#define KMX_PROFILE_KINDS 12
kmx_status kmx_profile_begin(kmx_space* sp, int capacity);
/* Bracket only the kinds whose bit is set in mask (bit k: kind k; default all
 * kinds) until kmx_profile_end.  Each bracketed launch is separated from
 * its neighbours by two event records; bracketing one kind leaves the
 * others' launches back to back. */
kmx_status kmx_profile_select(kmx_space* sp, unsigned mask);
kmx_status kmx_profile_end(kmx_space* sp, double* ms_total, int* launches);

/* ---- per-direction degrees, knot vectors and element counts -------------
 * Section 4.1: with a degree p_i and a knot vector Xi_i per direction i the
 * pairing blocks keep the Kronecker form of eqs. (4.2)/(4.3), each 1D factor
 * G^i, M^i built from the bases of direction i, and a solve stays one banded
 * 1D solve per axis (eqs. (4.4)-(4.5)).  A kmx_tspace holds the spaces of the
 * second scheme for such a mesh: direction a (0 = x, 1 = y, 2 = z) has degree
 * p[a] (2..4), n_elem[a] elements (n_elem[a] + p[a] - 1 <= 76) and a p-open
 * knot vector with the n_elem[a] - 1 interior breakpoints breaks_a (host,
 * strictly increasing inside (0, 1); NULL: uniform).  Map kinds 0 and 1 only
 * (host struct; kind 1 as for kmx_create_space).  Unknowns are laid out as in
 * the single-degree spaces: the three components one after the other, x
 * fastest inside; component c of a form space has, along direction a, the
 * univariate space of its tag (Section 2.3): for X^1_{h,0} (and X~^2) the
 * derivative space along c (dimension N_a + p_a - 1) and the value space across
 * it (N_a + p_a - 2); for X^2_{h,0} (and X~^1) the other way round.  Gauss
 * rules: p_a + 1 points per element and direction.  The metric factor is
 * streamed (6 doubles per quadrature point).  Errors: KMX_E_ARG (sizes,
 * degrees, breakpoints, map kind, a pairing factor that needs pivoting),
 * KMX_E_GEOMETRY, KMX_E_OOM, KMX_E_DEVICE.  Calls on one space must not
 * overlap (they share its scratch). */
typedef struct kmx_tspace kmx_tspace;
kmx_status kmx_create_tspace(const int* p, const int* n_elem, const double* breaks_x, const double* breaks_y,
                             const double* breaks_z, const kmx_map* map, int max_batch, kmx_tspace** out);
void kmx_destroy_tspace(kmx_tspace* ts);
/* n_e = dim X^1_{h,0} = dim X~^2, n_h = dim X~^1 = dim X^2_{h,0} (either may be NULL). */
kmx_status kmx_tspace_sizes(const kmx_tspace* ts, int64_t* n_e, int64_t* n_h);
/* Per-element eps and mu (host, N_x N_y N_z each, x fastest; NULL = 1).
 * Errors: KMX_E_MATERIAL (nothing changed), KMX_E_DEVICE. */
kmx_status kmx_tspace_set_materials(kmx_tspace* ts, const double* eps_elem, const double* mu_elem);
/* The form of the pairing solves (eqs. (4.4)-(4.5)): dense = 1 applies the
 * dense FP64 inverses of the 1D factors on the matrix cores (the default when
 * every line has at most 80 entries), dense = 0 the banded LU substitutions.
 * Same results up to rounding.  Errors: KMX_E_ARG; KMX_E_STATE for dense = 1
 * on a space with a longer line. */
kmx_status kmx_tspace_set_solver(kmx_tspace* ts, int dense);
/* The operators of one field (device vectors, as kmx_op_curl, kmx_op_mass
 * without the fused curl, kmx_op_solve and kmx_op_pairing). */
kmx_status kmx_tspace_op_curl(kmx_tspace* ts, int which, const double* x, double* y, void* stream);
kmx_status kmx_tspace_op_mass(kmx_tspace* ts, int which, const double* x, double* y, void* stream);
kmx_status kmx_tspace_op_solve(kmx_tspace* ts, int which, int transpose, const double* y, double* x,
                               void* stream);
kmx_status kmx_tspace_op_pairing(kmx_tspace* ts, int which, const double* x, double* y, void* stream);
/* nsteps source-free leapfrog steps (Section 3.4, as kmx_step):
 *   h -= dt K~1^{-1} M^2_{1/mu} D^1 e,  e += dt K1^{-1} M~^2_{1/eps} D~^1 h,
 * with b -= dt D^1 e and d += dt D~^1 h when flags has KMX_TRACK_DB (E holds
 * [e | d], H holds [h | b] per member); batch members back to back. */
kmx_status kmx_tspace_step(kmx_tspace* ts, double* E, double* H, double dt, int nsteps, int batch, int flags,
                           void* stream);

const char* kmx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
