/*
 * gks.h -- C ABI of the MI355X (gfx950) library for one two-stage fourth-order (S2O4) time step of the
 * high-order gas-kinetic scheme (GKS) for 3D weakly compressible isothermal flow on a structured
 * Cartesian grid (uniform, or stretched per axis: gks_config.faces), with actuator-line (ALM) and
 * immersed-boundary (IBM) body forces.
 *
 * Method: Huo, Pan, Cao, Meng, Tian, Huang, "High-order gas-kinetic scheme for numerical simulations
 * of wind turbine with nacelle and tower using ALM and IBM" (arXiv 2603.11102):
 *   Section 2      BGK model, isothermal Maxwellian, finite-volume form (Eqs. (semi), (finite),
 *                  (x_example)), interface distribution (Eq. (flux)), WENO reconstruction, S2O4, CFL dt;
 *   Appendix       microscopic coefficients of g0;
 *   Section 3.1    actuator line model (Eqs. (axial-tangential), (Gaussian));
 *   Section 3.2    direct-forcing immersed boundary (Eqs. (ibm-1), (force-ibm));
 *   Section 3.3    momentum update with the external body force after the S2O4 step;
 *   Section 4.4.1  power and thrust coefficients.
 *
 * Memory ownership: the CALLER owns every device buffer (fields, workspace, checkpoints, scalings)
 * and keeps it alive until gks_destroy. The library never allocates device memory; it holds a small
 * host context and one static device array per GPU (the workspace of gks_init_static, for callers
 * that cannot allocate). All device work is enqueued on the HIP stream given to gks_init, in order.
 *
 * Fields: a gks_field is four device pointers (rho - rho_ref, rho U, rho V, rho W). Each points to
 * (nx+6)(ny+6)(nz+6) elements of the configured precision (float or double), x fastest, then y, then
 * z, with 3 ghost layers per side: cell (i, j, k), -3 <= i < nx+3, sits at
 * ((k+3)(ny+6) + (j+3))(nx+6) + (i+3). Density is stored as its deviation from rho_ref.
 *
 * Errors: every call returns GKS_OK (0) or a GKS_E_* code and never throws across the ABI; the last
 * message of a context is available from gks_last_error. Contexts are not thread-safe.
 */
#ifndef GKS_H
#define GKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GKS_OK 0
#define GKS_E_INVALID_ARG 1   /* argument out of range, inconsistent sizes, null pointer */
#define GKS_E_STATE 2         /* call out of order (e.g. adjoint without a checkpoint window) */
#define GKS_E_HIP 3           /* a HIP runtime call failed */
#define GKS_E_NONFINITE 4     /* a non-finite value was found in the field (reported by gks_forces) */
#define GKS_E_UNSTABLE 5      /* |U|_max reached the sound speed (reported by gks_forces) */
#define GKS_E_UNSUPPORTED 6   /* valid request the library does not implement */
#define GKS_E_BODY_LEFT 7     /* a moving body's point support left the interior (reported by gks_forces) */

/* boundary kinds, per side, order x-, x+, y-, y+, z-, z+ */
#define GKS_BC_PERIODIC 0
#define GKS_BC_NOSLIP_WALL 1  /* mirror: rho even, all momenta odd (no-slip isothermal wall) */
#define GKS_BC_SLIP_WALL 2    /* mirror: normal momentum odd, rest even (slip / symmetry wall) */
#define GKS_BC_INFLOW 3       /* prescribed velocity u_in, rho from the outgoing isothermal Riemann invariant */
#define GKS_BC_OUTFLOW 4      /* zero-gradient extrapolation */

#define GKS_FP32 0
#define GKS_FP64 1

/* gks_forces_out.flags bits (warnings, non-fatal) */
#define GKS_WARN_EPS_SMALL 1  /* ALM eps < 2 dx (Section 4.3.1 advises eps >= 2 dx) */
#define GKS_WARN_MACH 2       /* Ma > 0.3: outside the weakly compressible regime */

typedef struct gks_config {
    int32_t nx, ny, nz;          /* interior cells per axis, each >= 3 */
    int32_t precision;           /* GKS_FP32 or GKS_FP64: storage and arithmetic of the stage kernels */
    double x0, y0, z0;           /* low corner of the domain */
    double lx, ly, lz;           /* domain lengths (uniform spacing lx/nx, ...) */
    double ma, u_ref;            /* lambda = ma^2 / (2 u_ref^2) (Section 2); sound speed sqrt(1/(2 lambda)) */
    double rho_ref;              /* reference density; fields store rho - rho_ref */
    double mu;                   /* dynamic viscosity; collision time tau = mu / p (Section 2) */
    double cfl;                  /* > 0: dt = cfl h_min / (|U|_max + C) each step (Section 2), h_min the
                                    smallest cell width */
    double dt_fixed;             /* used when cfl <= 0 (the constant dt of Section 4.3) */
    int32_t bc[6];               /* GKS_BC_* for x-, x+, y-, y+, z-, z+; periodic must be paired */
    double u_in[3];              /* inflow velocity for GKS_BC_INFLOW sides */
    double body_force[3];        /* constant body force G per unit volume, added as dt G after the step */
    double weno_eps;             /* WENO-JS epsilon (1e-6 if <= 0) */
    int32_t ibm_iters;           /* direct-forcing iterations per step (fixed count, >= 1) */
    int32_t max_act;             /* capacity of the workspace for actuator points (0 = no rotor), <= 1024 */
    int64_t max_ibm;             /* capacity of the workspace for Lagrangian points (0 = no bodies) */
    int32_t order;               /* 5 (or 0): the high-order GKS (fifth-order WENO-JS to 2x2 Gauss points,
                                    Section 2); 2: the second-order GKS of the comparison in Section 4.3.3
                                    (van Leer-limited linear face states, one flux point per face) */
    const double* faces[3];      /* NULL: uniform axis. Else HOST array of the n+1 increasing cell-face
                                    coordinates of a stretched axis (the channel of Section 4.1 is computed
                                    on a tanh-clustered mesh given by a coordinate transformation), with
                                    faces[0] = x0 and faces[n] = x0 + lx (relative 1e-12). Reconstruction
                                    runs in index space; derivatives take the local spacings (normal: the
                                    distance of the adjacent cell centres, the adjacent width at a boundary
                                    face; tangential: the line's cell width); the face flux is the mean of
                                    its Gauss-point fluxes times the face area; the CFL step takes the
                                    smallest width. Read during gks_init only. A periodic axis must be
                                    uniform. A rotor (its disc and 3 eps spheres) or an immersed body must
                                    sit in cells of one width (a uniformly refined block, as around the
                                    paper's turbines) and then works on the uniform grid of that block
                                    (a moving body on the widest run of cells of that width). */
} gks_config;

typedef struct gks_field {
    void* rho;  /* rho - rho_ref */
    void* mx;   /* rho U */
    void* my;   /* rho V */
    void* mz;   /* rho W */
} gks_field;

typedef struct gks_rotor {
    int32_t n_blades, n_per_blade;   /* actuator points: n_blades * n_per_blade, blade-major */
    double hub[3];                   /* rotor centre; the rotor axis is +x */
    double omega, theta0;            /* blade b at angle theta0 + omega t + 2 pi b / n_blades about +x */
    double radius;                   /* tip radius R (for C_P, C_T) */
    double u_inf;                    /* reference velocity of C_P, C_T */
    const double* r;                 /* host, n_per_blade: radius of each point */
    const double* chord;             /* host, n_per_blade */
    const double* twist;             /* host, n_per_blade: local twist gamma (rad) */
    const double* width;             /* host, n_per_blade: element width w */
    double eps;                      /* Gaussian smearing width (Eq. (Gaussian)), truncated at 3 eps */
    double cl_slope, alpha_clip;     /* synthetic polar C_L = cl_slope * clamp(alpha, +-alpha_clip) */
    double cd0, cd2;                 /* C_D = cd0 + cd2 alpha^2 (alpha in rad) */
    int32_t u_inf_correction;        /* 1: free-stream velocity correction of Section 3.1 */
    int32_t tip_correction;          /* 1: tip correction of Section 4.4, Eq. (tip-correction), on F_x and F_theta */
    const double* scale;             /* DEVICE, n_act doubles: per-point force scaling s_p; NULL = 1 */
    int32_t line_points;             /* line sampling of the NTNU rotor (Sections 3.1, 4.4; the method is
                                        defined in the work they cite, so this is a stated reading): the
                                        velocity of a point is the mean of trilinear samples at line_points
                                        points, the midpoints of equal parts of the segment of half-length
                                        line_half_length through it along the blade's direction of motion.
                                        <= 1 or a zero length: point sampling (Section 3.1, NREL rotor) */
    double line_half_length;         /* >= 0; every sampling segment must stay inside the interior cells */
} gks_rotor;

typedef struct gks_forces_out {
    double t, dt;                    /* time after the last step and its dt */
    int64_t step;                    /* steps taken since gks_init */
    double thrust, torque, power;    /* rotor loads of the last step (FP64 reductions) */
    double cp, ct;                   /* 2 P/(rho pi R^2 U^3), 2 T/(rho pi R^2 U^2) (Section 4.4.1) */
    double ibm_force[3];             /* total IBM force on the bodies, last step: -sum_s sum_cells F^s */
    double ibm_residual;             /* max_p |v_p - interpolated U| after the last iteration */
    int32_t ibm_iters_used;
    int32_t flags;                   /* GKS_WARN_* bits */
    double mass, mom[3];             /* interior sums of rho - rho_ref and rho U (times cell volume) */
    double umax;                     /* max |U| over interior cells */
    double window_power, window_thrust; /* sums of P and T over steps since the last window reset */
    int64_t window_steps;
    /* optional HOST arrays of n_act doubles, filled if non-NULL */
    double* alpha;
    double* fx;
    double* ftheta;
    double* urel;
} gks_forces_out;

/* Rigid motion of an immersed body: the body's points are at their given positions at time t0; the
 * centre c0 moves with the constant translation velocity, the body turns about the moving centre with
 * the constant angular velocity omega (rad per unit time, right-handed about omega). */
typedef struct gks_motion {
    double center[3];
    double velocity[3];
    double omega[3];
    double t0;
} gks_motion;

typedef struct gks_ctx gks_ctx;

/* Bytes of device workspace the caller must provide to gks_init for this configuration (including
 * room for cfg->max_act actuator points and cfg->max_ibm Lagrangian points). Returns 0 on invalid
 * input. */
size_t gks_workspace_bytes(const gks_config* cfg);

/* Create a context. q holds Q^0 (interior cells; ghosts are filled here), q_stage and q_acc are the
 * stage buffers (Q* and the S2O4 accumulator), same layout. workspace: device, >= the bytes above,
 * 256-byte aligned. hip_stream: a hipStream_t (NULL = default stream). Validates the configuration,
 * fills the ghost cells of q and enqueues nothing else. */
int gks_init(const gks_config* cfg, gks_field q, gks_field q_stage, gks_field q_acc, void* workspace,
             size_t workspace_bytes, void* hip_stream, gks_ctx** out);

/* Set (or replace) the rotor of the actuator line model (Section 3.1). Host arrays are copied; the
 * device scale array is referenced and read at every step. Every actuator point, its sampling cells
 * and its 3 eps projection sphere must lie inside the interior cells. GKS_E_UNSUPPORTED on a stretched
 * mesh when these cells do not share one width per axis. */
int gks_set_actuators(gks_ctx* ctx, const gks_rotor* rotor);

/* Set the Lagrangian points of the immersed bodies (Section 3.2): n points at fixed positions, host
 * xyz [n][3], surface areas dS [n] and velocities vel [n][3] (NULL: stationary points, the paper's
 * nacelle and tower). Each point's 4x4x4 discrete-delta support must lie inside the interior cells.
 * Computes on the device the interpolated volumes V-bar = sum W V_p (V_p = dx dS_p) and cell
 * velocities v-bar = sum W V_p v_p / V-bar that the forcing drives the fluid towards. Host arrays
 * are copied; GKS_E_INVALID_ARG for bad sizes, points or values; GKS_E_UNSUPPORTED on a stretched mesh
 * when the cells within two cells of the body do not share one width per axis. */
int gks_set_ibm_points(gks_ctx* ctx, int64_t n, const double* xyz, const double* dS, const double* vel);

/* Move the body of the last gks_set_ibm_points rigidly (the introduction and Section 3.2 have the
 * Lagrangian points follow the body's translation and rotation; the paper's own bodies are at rest).
 * The points given there are the positions at motion->t0. From the next step on, every step from t^n
 * to t^{n+1} places each point at X_p = c + R(omega (t^{n+1} - t0)) (X_p(t0) - c0), c = c0 +
 * velocity (t^{n+1} - t0), gives it the velocity v_p = velocity + omega x (X_p - c) (replacing the
 * velocities of gks_set_ibm_points) and rebuilds the supports, V-bar and v-bar on the device before
 * the forcing; nothing is synchronised and nothing allocated. The motion lasts until the next
 * gks_set_ibm_points. If a point's 4x4x4 support leaves the interior cells (on a stretched mesh: the
 * run of cells of the body's width around its initial position) the forcing stops for that and every
 * later step and gks_forces returns GKS_E_BODY_LEFT. Returns GKS_E_STATE without points,
 * GKS_E_INVALID_ARG for a null or non-finite motion. */
int gks_set_ibm_motion(gks_ctx* ctx, const gks_motion* motion);

/* Enqueue nsteps S2O4 steps (Section 2) with the body-force update of Section 3.3 on the stream and
 * return without synchronising. dt stays on the device. */
int gks_step(gks_ctx* ctx, int32_t nsteps);

/* Synchronise the stream and report the FP64 loads, coefficients, conservation sums and time of the
 * last step. Returns GKS_E_NONFINITE / GKS_E_UNSTABLE (after filling out) when the field is not finite
 * or |U|_max >= sound speed. */
int gks_forces(gks_ctx* ctx, gks_forces_out* out);

/* Reset the window sums of power and thrust (gks_forces_out.window_*). Enqueued on the stream. */
int gks_reset_window(gks_ctx* ctx);

/* FP32 contexts carry the state as the field q plus a low-order part held in the workspace (the
 * S2O4 stage updates of Section 2 are applied as error-free sums, so the stored state keeps about
 * twice the FP32 digits across steps while every flux is still evaluated from q in FP32). A caller
 * that overwrites q after gks_init must call this before the next gks_step: it clears the low-order
 * part (enqueued on the stream). FP64 contexts: no effect. Returns GKS_E_INVALID_ARG for a null ctx,
 * GKS_E_HIP if the clear cannot be enqueued. */
int gks_field_changed(gks_ctx* ctx);

/* Bytes of device memory one checkpoint slot needs: three fields of a step (Q^n, the S2O4 intermediate
 * state Q* and the field before the body forces of Section 3.3) and its time. */
size_t gks_checkpoint_slot_bytes(const gks_config* cfg);

/* Register a DEVICE buffer of `capacity` checkpoint slots (or NULL to stop); the window sums are reset.
 * While registered, every gks_step stores in slot (window step index) Q^n (before the step), Q* and the
 * field before the body forces. Used by gks_adjoint to run each step backwards. */
int gks_set_checkpoints(gks_ctx* ctx, void* buffer, int32_t capacity);

/* Bytes of device scratch gks_adjoint needs. */
size_t gks_adjoint_workspace_bytes(const gks_config* cfg, int32_t n_act);

/* gks_adjoint flags */
#define GKS_ADJ_EXACT_WENO 1  /* differentiate the WENO nonlinear weights too (default: frozen) */

/* Reverse-mode gradient of J = w[0] * mean_n P^n + w[1] * mean_n T^n over the first nsteps
 * checkpointed steps of the window with respect to the per-point force scalings s_p, written to grad_s
 * (DEVICE, n_act doubles, overwritten). If grad_q0 is not NULL it receives dJ/dQ^0 (DEVICE, 4 arrays of
 * nx*ny*nz doubles back to back, interior cells, x fastest; variable 0 is the density). By default the
 * WENO nonlinear weights are frozen at their forward values (differentiated as constants); with
 * GKS_ADJ_EXACT_WENO in flags they are differentiated as well, so the gradient is the derivative of the
 * discrete forward itself. Everything else (flux, kinetic average, S2O4 combination, ghost cells,
 * actuator-line sampling, forces and projection, the direct forcing of an immersed body at rest) is
 * linearised exactly, as are the ghost cells of every boundary kind (the inflow's Riemann-invariant
 * density at the stage's field), on a uniform or a stretched mesh (the chain-rule derivatives and flux
 * differences carry the local spacings). Requires an FP64 context of the high-order scheme (order 5)
 * with a rotor, no moving body and a fixed dt. The stage buffers q_stage and q_acc are overwritten; q
 * is not. adj_ws: device scratch of
 * gks_adjoint_workspace_bytes (256-byte aligned). Synchronises the stream. */
int gks_adjoint(gks_ctx* ctx, int32_t nsteps, const double w[2], double* grad_s, double* grad_q0,
                void* adj_ws, size_t adj_ws_bytes, int32_t flags);

/* Running flow statistics of the cell velocity U = (rho U)/rho (Sections 4.1, 4.2, 4.3.2). The caller
 * provides a DEVICE buffer of gks_statistics_bytes (8-byte aligned); gks_set_statistics clears it and
 * from then on every `interval`-th step adds a sample (mean and co-moments updated per cell in FP64).
 * NULL disables. */
size_t gks_statistics_bytes(const gks_config* cfg);
int gks_set_statistics(gks_ctx* ctx, void* buffer, int32_t interval);

/* Enqueue the statistics of the samples so far into DEVICE arrays (each may be NULL; interior cells,
 * x fastest): mean [3][n] (U, V, W), rms [3][n] = sqrt(<U'^2>) etc., stress [3][n] = <U'V'>, <U'W'>,
 * <V'W'>, tke [n] = (<U'^2> + <V'^2> + <W'^2>) / (2 u_inf^2), with n = nx*ny*nz; nsamples (host) gets
 * the sample count. */
int gks_read_statistics(gks_ctx* ctx, double u_inf, double* mean, double* rms, double* stress, double* tke,
                        int64_t* nsamples);

/* Per-step load history (the C_P / C_T time histories of Section 4.4.1): each step appends 10 doubles
 * (t, dt, thrust, torque, power, C_P, C_T, IBM force x, y, z) to the DEVICE buffer until `capacity`
 * records are written. NULL disables. gks_history_count returns the records written. */
int gks_set_history(gks_ctx* ctx, double* buffer, int32_t capacity);
int gks_history_count(gks_ctx* ctx, int64_t* count);

/* Per-launch timing with HIP events recorded on the context's stream around each launch group.
 * Categories (index into the arrays of gks_read_timing): */
#define GKS_TIMER_GHOST 0      /* ghost-cell fills (3 launches per stage) */
#define GKS_TIMER_DT 1         /* |U|max reduction and the dt update */
#define GKS_TIMER_S1X 2        /* stage-1 face kernel, x faces */
#define GKS_TIMER_S1Y 3
#define GKS_TIMER_S1Z 4        /* includes the stage-1 S2O4 combination */
#define GKS_TIMER_S2X 5        /* stage-2 face kernel, x faces */
#define GKS_TIMER_S2Y 6
#define GKS_TIMER_S2Z 7        /* includes the final combination and the constant body force */
#define GKS_TIMER_ALM 8
#define GKS_TIMER_IBM 9
#define GKS_TIMER_OTHER 10     /* checkpoint copies and step bookkeeping */
#define GKS_TIMER_COUNT 11

/* Enable (1) or disable (0) event timing; enabling clears the accumulated totals. Host-side event
 * objects are created on demand (no device memory). */
int gks_set_timing(gks_ctx* ctx, int32_t enable);

/* Synchronise the stream and return the accumulated milliseconds and launch-group counts per
 * category (arrays of n <= GKS_TIMER_COUNT entries). */
int gks_read_timing(gks_ctx* ctx, double* ms, int64_t* count, int32_t n);

/* Bytes of the library's static device scratch (one array per GPU, held until the process ends). */
#define GKS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): gks_init with the workspace taken from the library's static device
 * array of GKS_STATIC_SCRATCH_BYTES on the current device (which must be the stream's). Allocates no
 * device memory; the caller still provides q, q_stage and q_acc. Returns GKS_E_INVALID_ARG when
 * gks_workspace_bytes(cfg) exceeds GKS_STATIC_SCRATCH_BYTES (e.g. FP32 grids above about 64^3, FP64
 * above about 48^3, or room for many Lagrangian points), and GKS_E_STATE while another context made
 * here on the same GPU is alive: one GPU holds one such workspace, and it keeps the last context's
 * contents (gks_init_static clears what must start at zero). Contexts made by gks_init are not affected.
 * The context is used and destroyed like any other; gks_destroy releases the scratch. */
int gks_init_static(const gks_config* cfg, gks_field q, gks_field q_stage, gks_field q_acc, void* hip_stream,
                    gks_ctx** out);

/* Release the host context (device buffers stay the caller's). */
void gks_destroy(gks_ctx* ctx);

/* Last error message of a context (or of the last failed gks_init when ctx is NULL). */
const char* gks_last_error(const gks_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GKS_H */
