/*
 * adjoint.h -- C ABI of the per-time-step analytical adjoint for Neo-Hookean
 * tet meshes with smoothed Fischer-Burmeister frictional contact
 * ("Fast and Reliable Gradients for Deformables Across Frictional Contact
 * Regimes", arXiv 2603.16478).  One GPU (gfx950), HIP.
 *
 * Problem statement (Sec. 3, eq:implicit, eq:lagrange, eq:contact,
 * eq:internal, eq:dynamics): an implicit step maps (qbar, vbar, f_ext;
 * E, nu, mu) to (q, v).  Its adjoint (Sec. 5.1, eq:adjoint) solves
 *     Acal^T z = (dL/dq + dL/dv / h)^T,   Acal = A - dA + h^2 H_c^T K_c H_c
 * and maps z to gradients (eq:compute_gradient, App. B.3).
 *
 * Conventions for every entry point
 *   - Arrays marked "device" are device pointers (HIP global memory) owned
 *     by the caller; arrays marked "host" are host memory read during the
 *     call.  Vectors over vertices are AoS [n_verts][3] double.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Calls enqueue work and may return before it finishes, except
 *     where stated.  Outputs are valid after the stream synchronises.
 *   - Every call returns an adj_status.  On error nothing is enqueued (shape
 *     and argument errors are detected before any launch) and
 *     adj_last_error() returns a message (thread-local).
 *   - A scene is used by one host thread at a time.
 */
#ifndef PAPER_2603_16478_ADJOINT_H
#define PAPER_2603_16478_ADJOINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADJ_OK = 0,
  ADJ_E_ARG = -1,       /* null pointer, non-finite or out-of-range argument */
  ADJ_E_SHAPE = -2,     /* sizes inconsistent with the scene */
  ADJ_E_INVERTED = -3,  /* a tet with det F <= 0 (Neo-Hookean log J undefined) */
  ADJ_E_NOCONV = -4,    /* Krylov / Newton did not reach the tolerance; outputs hold the last iterate */
  ADJ_E_SINGULAR = -5,  /* zero or non-finite pivot (elastic factor or capacitance) */
  ADJ_E_DEVICE = -6,    /* a HIP runtime call failed */
  ADJ_E_OOM = -7,       /* device or host allocation failed */
  ADJ_E_NOTIMPL = -8
} adj_status;

/* ADJ_MIXED: iterative refinement, FP64 residual b - Acal^T z, inner GMRES
 * (or PCG) with FP32 block values, FP32 sparse inverse or sweeps and FP64
 * Woodbury factors.  ADJ_MIXED_PC: one FP64 flexible GMRES whose
 * preconditioner applies the sparse inverse (or the sweeps) in FP32; the
 * product, Gram-Schmidt and residual stay FP64 (PCG solves and batches take
 * it as ADJ_MIXED). */
typedef enum { ADJ_FP64 = 0, ADJ_MIXED = 1, ADJ_MIXED_PC = 2 } adj_precision;

typedef struct adj_scene adj_scene; /* opaque */

/* Material model of the local projection step (App. B.2): the singular
 * values theta of the projected F minimise w/2 |theta - sigma|^2 + zeta(theta)
 * with w = 2 mu.  Neo-Hookean: zeta from the stable Neo-Hookean energy
 * (Newton on the optimality condition); ARAP: theta = 1 (the projection is
 * the rotation of F, W = 0); co-rotational: zeta = mu |theta - 1|^2 +
 * lam/2 (sum(theta - 1))^2 (linear optimality condition, constant W).  A
 * batch's scenes share the model. */
typedef enum { ADJ_MAT_NEO_HOOKEAN = 0, ADJ_MAT_ARAP = 1, ADJ_MAT_COROT = 2 } adj_material;

/* Scene description (host memory, read during adj_scene_create only).
 * Mesh and material (Sec. 3.1, 3.3): rest positions, tets with positive
 * orientation, density, Young's modulus E and Poisson ratio nu (scalars, or
 * one value per tet when per_tet_material = 1).  Contact colliders: planes
 * (n, d) with gap n.x - d, unit n.  h = time step, eps = smoothing parameter
 * of phi_eps(x,y) = x + y - sqrt(x^2 + y^2 + 2 eps^2) (Sec. 5.2).
 * Bilateral bindings (Sec. 3.2 eq:binding): vertex binding_vid[b] is held to
 * a target d_b, given per step (adj_binding_vjp), by a linear spring of
 * compliance binding_E[b] > 0; the vertices are distinct.  The binding term
 * h^2 J_b^T E_b^{-1} J_b is constant, so it is part of the prefactored system
 * matrix A.  Leave n_bindings = 0 (zero-initialised description) for none. */
typedef struct {
  int32_t n_verts;
  int32_t n_tets;
  const double* rest_pos; /* host [n_verts*3] */
  const int32_t* tets;    /* host [n_tets*4] */
  double density;
  double h;
  double eps;
  const double* E;        /* host [1] or [n_tets] */
  const double* nu;       /* host [1] or [n_tets] */
  int32_t per_tet_material;
  double gravity[3];
  int32_t n_planes;
  const double* planes;   /* host [n_planes*4] */
  double contact_margin;  /* candidate if predicted gap <= margin */
  int32_t n_bindings;
  const int32_t* binding_vid; /* host [n_bindings] */
  const double* binding_E;    /* host [n_bindings] */
  int32_t material;           /* adj_material; 0 (zero-initialised) = Neo-Hookean */
} adj_scene_desc;

/* Converged contact state of one step (the forward step record).  All
 * arrays are device memory, n_contacts entries, sorted by vertex id.
 * frame: rows (n, t1, t2) of the contact frame H_c (Sec. 3.2); delta and
 * lambda: delta_c and lambda_c in frame coordinates (delta_n, delta_f1,
 * delta_f2), (lambda_n, lambda_f1, lambda_f2).  fric = 1 for a contact with
 * friction rows, 0 for a normal-only contact.  d_n, d_f: offsets of the
 * constraint (delta_n = n.x - d_n, delta_f = T (x - xbar) - d_f). */
typedef struct {
  int32_t n_contacts;  /* host value */
  int32_t capacity;    /* host value: allocated entries (forward output only) */
  int32_t* vid;        /* device [capacity] */
  int32_t* fric;       /* device [capacity] */
  double* frame;       /* device [capacity*9] */
  double* delta;       /* device [capacity*3] */
  double* lambda;      /* device [capacity*3] */
  double* d_n;         /* device [capacity] */
  double* d_f;         /* device [capacity*2] */
  double mu;           /* friction coefficient of the step */
} adj_contact_state;

/* Krylov method (Sec. 5.4: GMRES for the non-symmetric frictional system,
 * conjugate gradients when the system is symmetric positive definite).
 * ADJ_AUTO picks PCG when no contact is frictional or mu = 0 (then every
 * contact block, hence Acal^T and the Woodbury preconditioner, is symmetric),
 * GMRES otherwise; ADJ_PCG on a non-symmetric system is ADJ_E_ARG. */
/* ADJ_SEMI_IMPLICIT (single-scene FP64 solves): the fixed-point iteration
 * x <- x + A^{-1} (b - Acal^T x) of the semi-implicit baselines the paper
 * compares against (Sec. 6.2); it converges only while the spectral radius
 * of I - A^{-1} Acal^T stays below one and is reported as ADJ_E_NOCONV
 * (outputs: the last iterate) when it does not reach the tolerance or
 * grows past 1e6 |b|. */
typedef enum { ADJ_AUTO = 0, ADJ_GMRES = 1, ADJ_PCG = 2, ADJ_SEMI_IMPLICIT = 3 } adj_krylov;

/* Preconditioner of the Krylov solve (single-scene calls; batches use the
 * Woodbury one).  ADJ_PRECOND_WOODBURY: A^{-1} = S^T S with the contact
 * blocks through the Woodbury identity (Sec. 5.4, the paper's choice);
 * ADJ_PRECOND_SPARSE_INVERSE: S^T S alone (the contact blocks are left to
 * the Krylov method); ADJ_PRECOND_JACOBI: the inverses of the 3x3 diagonal
 * blocks of Acal^T; ADJ_PRECOND_POINT_JACOBI: the inverse of its diagonal.
 * These are the comparison preconditioners of the paper's backward-solver
 * study (Sec. 6.2); all give the same solution to the tolerance.
 * ADJ_PRECOND_WOODBURY_NO_Z: the Woodbury preconditioner with its correction
 * A^{-1} H^T t applied by two more sparse-inverse products per apply instead
 * of the cached dense Z = A^{-1} H^T.  ADJ_PRECOND_WOODBURY switches to this
 * form by itself when forming Z would cost more than 2e10 multiply-adds
 * (nnz(S) x contact vertices; the slab workload). */
typedef enum {
  ADJ_PRECOND_WOODBURY = 0,
  ADJ_PRECOND_SPARSE_INVERSE = 1,
  ADJ_PRECOND_JACOBI = 2,
  ADJ_PRECOND_POINT_JACOBI = 3,
  ADJ_PRECOND_WOODBURY_NO_Z = 4
} adj_precond;

typedef struct {
  double rtol;          /* relative residual |b - Acal^T z| / |b| (Sec. 6.1: 1e-8) */
  int32_t maxit;        /* total Krylov iterations over all restarts */
  int32_t restart;      /* GMRES restart length, 1..128 */
  int32_t max_refine;   /* outer refinement sweeps: mixed precision (FP64
                         * residual, FP32-stored inner solves); FP64 with
                         * rtol below 1e-9 (residual summed in double-double,
                         * FP64 inner solves to 1e-9, since plain FP64 Krylov
                         * stagnates near there on stiff contacts); 0 turns
                         * FP64 refinement off */
  adj_precision prec;
  int32_t reuse_delassus; /* 1: keep H A^{-1} H^T while the contact vertex set is unchanged */
  adj_krylov method;
  adj_precond precond;  /* 0 (zero-initialised options): Woodbury */
} adj_solve_opts;

typedef struct {
  int32_t iters;        /* Krylov iterations taken */
  int32_t refine_steps;
  int32_t n_contacts;
  int32_t m_rows;       /* rows of the contact-space capacitance */
  double relres;        /* true relative residual at exit */
  int32_t delassus_rebuilt;
  int32_t method;       /* ADJ_GMRES or ADJ_PCG: the method that ran */
} adj_solve_info;

/* Build the scene: rest-shape operators, lumped mass, the constant system
 * matrix A = M + h^2 sum_i w_i G_i^T G_i (eq:dynamics) and its Cholesky
 * factor with its sparse inverse S = L^{-1} (Sec. 3.4: A^{-1} = S^T S),
 * the block-sparse pattern of Acal with the element-to-entry map (Sec. 5.4,
 * matrix assembly), and device workspaces sized for `max_contacts`
 * (0 .. 10000; the capacitance inverse is dense, (3 max_contacts)^2 doubles).
 * Errors: ADJ_E_ARG, ADJ_E_INVERTED (rest tet with det <= 0),
 * ADJ_E_SINGULAR, ADJ_E_OOM, ADJ_E_DEVICE.  *out is NULL on error. */
adj_status adj_scene_create(const adj_scene_desc* desc, int32_t max_contacts, adj_scene** out);
adj_status adj_scene_destroy(adj_scene* scene);

/* Linearise the converged step (Sec. 5.2-5.4): per-tet SVD projection
 * Jacobians J_i (Sec. 5.3, App. B.0-B.4) assembled into the block-sparse
 * Acal^T through the element-to-entry map, contact blocks K_c, k_mu
 * (eq:final_diff_contact, App. A.1), and the Woodbury capacitance
 * K^{-T} + h^2 H A^{-1} H^T with its inverse (eq:woodbury_formula).
 * q: device [n_verts*3] converged positions.  The contact state must stay
 * alive and unchanged until adjoint_solve and vjp_params have run.
 * Errors: ADJ_E_SHAPE (n_contacts > max_contacts), ADJ_E_ARG.  Errors
 * found on the device (ADJ_E_INVERTED: a tet with det F <= 0, whose blocks
 * are then zero; ADJ_E_SINGULAR: a zero or non-finite capacitance pivot)
 * raise a flag that this call clears first; they are returned by the next
 * adjoint_solve (or adj_check_status) of the same scene. */
adj_status adjoint_setup(adj_scene* scene, const adj_contact_state* contacts, const double* q,
                         const adj_solve_opts* opts, void* stream);

/* Solve Acal^T z = dL_dq + dL_dv / h with right-preconditioned GMRES and
 * the Woodbury preconditioner (Sec. 5.4).  dL_dq, dL_dv: device
 * [n_verts*3]; z: device [n_verts*3] output.  Synchronises the stream at
 * the end (the iteration count and residual are host values).  Returns
 * ADJ_E_INVERTED or ADJ_E_SINGULAR when the last adjoint_setup raised that
 * device flag (z is then meaningless), else ADJ_E_NOCONV if rtol was not
 * met within maxit (z holds the last iterate), ADJ_E_SINGULAR for a
 * non-finite residual. */
adj_status adjoint_solve(adj_scene* scene, const double* dL_dq, const double* dL_dv, double* z,
                         const adj_solve_opts* opts, adj_solve_info* info, void* stream);

/* Gradients from z (eq:compute_gradient, App. B.3):
 *   dL_dqbar = M z + h^2 sum_c H_c^T P_f K_c^T H_c z - dL_dv / h
 *   dL_dvbar = h M z,   dL_dfext = h^2 z
 *   grad3[0] += dL/dE, grad3[1] += dL/dnu, grad3[2] += dL/dmu (friction)
 *   dE_tet[i] += dL/dE_i, dnu_tet[i] += dL/dnu_i (optional, may be NULL)
 * All pointers device; vectors [n_verts*3]; grad3 [3]; per-tet [n_tets].
 * Requires adjoint_setup on the same step. */
adj_status vjp_params(adj_scene* scene, const double* z, const double* dL_dv, double* dL_dqbar,
                      double* dL_dvbar, double* dL_dfext, double* grad3, double* dE_tet,
                      double* dnu_tet, void* stream);

/* vjp_params for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, kernels and results (bitwise), but its reduction
 * partials use a fixed device array of the library (512 KiB per device,
 * held until the process ends) instead of the scene's workspace; no call
 * allocates or frees memory.  The array's device address is looked up once
 * per device, on the first call with that device current.  Calls on one
 * device share the array: calls that overlap on one device (concurrent
 * streams or threads) race.  ADJ_E_SHAPE when the scene needs more than the
 * array holds (ceil(n_contacts/256) + 2 ceil(n_tets/256) > 65536 partial
 * sums, about 8.3 million tets). */
adj_status vjp_params_noalloc(adj_scene* scene, const double* z, const double* dL_dv, double* dL_dqbar,
                              double* dL_dvbar, double* dL_dfext, double* grad3, double* dE_tet,
                              double* dnu_tet, void* stream);

/* One implicit step (eq:dynamics): converge (q, lambda) from (qbar, vbar,
 * f_ext) with a damped Newton method whose linear systems are Acal du = r
 * (the adjoint matrix at the iterate, solved with the same GMRES and
 * Woodbury preconditioner), and write q, v and the contact state of the
 * step.  qbar, vbar, f_ext, q, v: device [n_verts*3]; f_ext excludes gravity
 * (taken from the scene).  contacts->capacity bounds the number of contacts
 * (ADJ_E_SHAPE beyond); its arrays receive the step record (d_n, d_f may be
 * NULL).  Contact multipliers are warm-started from the previous call on the
 * same scene (adj_forward_reset clears them).  Synchronises the stream.
 * Invalidates the last adjoint_setup.  Returns ADJ_E_NOCONV if the paper's
 * residual rows did not fall below 1e-8, ADJ_E_INVERTED for an inverted
 * element at the initial guess.  Scenes with bindings include the binding
 * forces at the targets of adj_set_binding_targets (ADJ_E_ARG if unset). */
adj_status sim_forward_step(adj_scene* scene, const double* qbar, const double* vbar,
                            const double* f_ext, double mu, double* q, double* v,
                            adj_contact_state* contacts, void* stream);

/* out[0] = Newton iterations of the last sim_forward_step, out[1] = the
 * max-norm of its residual rows (force rows in N, contact rows unscaled).
 * out: host [2]. */
adj_status adj_forward_stats(const adj_scene* scene, double* out);

/* Forget the warm start of the contact multipliers. */
adj_status adj_forward_reset(adj_scene* scene);

/* Binding targets d_b of the following sim_forward_step calls (Sec. 3.2
 * eq:binding): host [n_bindings * 3], in the order of the scene's bindings;
 * copied (synchronous).  A scene with bindings needs them before its first
 * forward step (ADJ_E_ARG otherwise); each forward step then adds the
 * binding force -(q_v - d_b) / E_b of every bound vertex.  ADJ_E_ARG for a
 * scene without bindings or a non-finite target. */
adj_status adj_set_binding_targets(adj_scene* scene, const double* targets);

/* Kinematic sphere colliders of the next sim_forward_step calls (the slab
 * workload's indenter): n spheres, old_pose and new_pose host [n][4] =
 * (centre x, y, z, radius) at the start and the end of the step.  A vertex
 * meets sphere s on the plane with normal n = (qbar_v - c_old)/|qbar_v -
 * c_old| and offset n . c_new + r_new, frozen for the step (Sec. 5.2); the
 * tangential motion of the sphere enters the friction displacement.  Spheres
 * count after the planes as colliders (at most 15 together).  n = 0 removes
 * them.  Copies the poses to the device (synchronously). */
adj_status adj_set_spheres(adj_scene* scene, int32_t n, const double* old_pose, const double* new_pose);

/* Actuation by active stress (the actuated-body workloads): tet t belongs to
 * group group[t] (host [n_tets], 0 .. n_groups-1) and has the fibre
 * direction fibre[t] (host [n_tets][3]); with the group parameters a (Pa) it
 * carries the first Piola stress a_g d d^T, whose nodal forces are
 * f_v = -V_t a_g (d d^T) grad N_v.  The force is linear in a: f = Phi a.
 * Copies the tables to the device (synchronises it). */
adj_status adj_set_actuation(adj_scene* scene, int32_t n_groups, const int32_t* group, const double* fibre);

/* f = Phi a: a device [n_groups], f device [n_verts*3] (overwritten), to be
 * passed to sim_forward_step as (part of) the external force. */
adj_status adj_actuation_force(adj_scene* scene, const double* a, double* f, void* stream);

/* dL/da = Phi^T dL/df: dL_df device [n_verts*3] (the step's dL/df_ext from
 * vjp_params), dL_da device [n_groups] (overwritten; fixed-order sums). */
adj_status adj_actuation_vjp(adj_scene* scene, const double* dL_df, double* dL_da, void* stream);

/* Scene sizes and host-side statistics: out[0] n_verts, out[1] n_tets,
 * out[2] nnz blocks of Acal, out[3] nnz(L), out[4] nnz(S), out[5]
 * max_contacts.  out: host [6]. */
adj_status adj_scene_info(const adj_scene* scene, int64_t* out);

/* Synchronise the stream and report device-side errors of the last setup
 * (ADJ_E_INVERTED when a tet had det F <= 0, ADJ_E_SINGULAR for a zero or
 * non-finite capacitance pivot).  The flag is cleared by the next setup. */
adj_status adj_check_status(adj_scene* scene, void* stream);

/* Diagnostics: copy an internal array of the last adjoint_setup to host
 * memory (synchronises the device).  what = 0: Acal^T block values
 * [nnz_blocks][3][3] row-major; 1: block row pointer [n_verts+1] int32;
 * 2: block column indices [nnz_blocks] int32; 3: inverse of the Woodbury
 * capacitance [mp][mp] (m rows padded with identity to mp, a multiple of
 * 64), or, when the capacitance took the block LU (tuning lu_min), its
 * factors in place of C, C = L D V with L unit block-lower, V unit
 * block-upper (128 x 128 blocks) and D = diag(U_KK), rewritten for the
 * grouped substitutions: per group of 4 consecutive diagonal blocks, the
 * strictly lower and strictly upper blocks inside the group hold the
 * inverses of the group's unit lower and unit upper parts, the lower blocks
 * below the group L_iG times the first, the upper blocks above it V_iG times
 * the second, diagonal blocks unused; 4: Delassus matrix of the contact
 * vertices [n_cv][n_cv];
 * 5: per-contact rotated bases Q = R frame [n_contacts][3][3]; 6: the
 * inverted diagonal blocks U_KK^{-1} of the block LU [mp/128][128][128]
 * (size 0 when the explicit inverse is in use).
 * *size_bytes receives the array size; nothing is copied when capacity_bytes
 * is smaller (ADJ_E_SHAPE).  For tests and debugging. */
adj_status adj_debug_export(const adj_scene* scene, int32_t what, void* host_out, int64_t capacity_bytes,
                            int64_t* size_bytes);

/* Binding gradients of the last adjoint_setup's step (Sec. 5.1
 * eq:differential_2, rhs_d_b and rhs_E_b): with z from adjoint_solve, q the
 * converged state and targets the step's binding targets d_b (device
 * [n_bindings][3]), writes dL/dd_b = h^2 z_b / E_b (device [n_bindings][3])
 * and dL/dE_b = -h^2 (lambda_b . z_b) / E_b with lambda_b = -(q_b - d_b) / E_b
 * (device [n_bindings]).  A scene without bindings returns ADJ_OK at once. */
adj_status adj_binding_vjp(adj_scene* scene, const double* z, const double* q, const double* targets,
                           double* dL_dtargets, double* dL_dE, void* stream);

/* Live timing of one kernel class: after adj_profile_begin(scene, kernel),
 * every launch of that kernel made by this scene's calls is bracketed by HIP
 * events on the stream it is launched on; adj_profile_end synchronises and
 * returns the summed kernel time (ms) and the launch count, then disarms.
 * kernel: 0 = S product (or the forward L sweeps), 1 = S^T product (or the
 * transposed sweeps), 2 = capacitance solve (inverse product, or the
 * block-LU substitutions),
 * 3 = Woodbury correction (Z product, or without Z the scatter and Y
 * product), 4 = block-sparse Acal^T product (in the Krylov loop fused
 * with the first Gram-Schmidt dots), 5 = per-tet Jacobian blocks, 6 = gather
 * assembly, 7 = the whole capacitance inversion or factorisation, 8 = second Gram-Schmidt
 * update with the Givens step, 9 = first Gram-Schmidt update, 10 = one
 * narrow Gauss-Jordan block step of the capacitance inversion, 11 = the
 * Delassus product (Y, D = Y^T Y and Z when cached), 12 = one trailing
 * update launch of the block-LU capacitance factorisation.  At most 65536
 * bracketed regions are timed per profile (later ones are not). */
adj_status adj_profile_begin(adj_scene* scene, int32_t kernel);
adj_status adj_profile_end(adj_scene* scene, double* total_ms, int64_t* launches);

/* Launch shapes of the Krylov loop.  They change only how work is split
 * over the GPU and the order of floating-point sums inside reductions (so
 * results are bitwise reproducible for a fixed tuning, and agree across
 * tunings to rounding).  Defaults: gs_rows 64, bsr_lanes 16, chunk 8,
 * graph 0, gj_wide_min 2048, a_inv 0, lu_min 4608, lu_pipe 1, sweep_fuse 0. */
typedef struct {
  int32_t gs_rows;   /* rows per 256-thread block of the Gram-Schmidt kernels: 64, 128, 256 */
  int32_t bsr_lanes; /* lanes per block row of the Acal^T product: 4, 8, 16, 32 */
  int32_t chunk;     /* Krylov iterations enqueued between host checks: 1..64 */
  int32_t graph;     /* 1: each chunk is captured once per setup as a HIP graph and replayed */
  int32_t gj_wide_min; /* padded capacitance size (a multiple of 128, >= 128) from which its inverse
                          runs the wide Gauss-Jordan steps (128 pivot columns per step) instead of
                          the 32-column ones; default 2048 */
  int32_t a_inv;     /* A^{-1} in the preconditioner: 1 = the sparse-inverse products S^T S, 2 = level-
                        scheduled sweeps with the Cholesky factor L, 0 = automatic (sweeps when S holds
                        more than 32 million and more than 4 nnz(L) entries) */
  int32_t lu_min;    /* padded capacitance size (a multiple of 128, >= 128) from which the capacitance
                        is factored by block LU (2/3 mp^3 on the matrix cores; each apply two block
                        substitutions) instead of inverted explicitly (2 mp^3; each apply one dense
                        product); default 4608 */
  int32_t lu_pipe;   /* 1: the block-LU substitutions run pipelined, one launch per pass (stripes of 16
                        rows that wait for the values they need, published once each by atomic stores);
                        0: one launch per group of four 128-blocks; default 1 */
  int32_t sweep_fuse; /* the lowest levels of each sweep with L run as one launch, one block per
                         independent part (the rows that those levels couple): that many levels, 0 =
                         none, -1 = automatic (the most levels that still split into at least 256
                         parts); default 0 */
} adj_tuning;

/* Set or read the scene's launch shapes.  ADJ_E_ARG on a value outside the
 * listed sets. */
adj_status adj_set_tuning(adj_scene* scene, const adj_tuning* t);
adj_status adj_get_tuning(const adj_scene* scene, adj_tuning* t);

/* Autotuner: after adjoint_setup, times adjoint_solve with right-hand side
 * (dL_dq, dL_dv) under candidate launch shapes (coordinate descent over
 * gs_rows, bsr_lanes, chunk and graph, each candidate the best of `reps`
 * timed solves, HIP events on `stream`), keeps the fastest on the scene and
 * writes it to *best (host).  z: device scratch [n_verts*3] that receives
 * the last solution.  Synchronises the stream. */
adj_status adj_autotune(adj_scene* scene, const double* dL_dq, const double* dL_dv, double* z,
                        const adj_solve_opts* opts, int32_t reps, adj_tuning* best, void* stream);

/* ---- Batched solves: many independent scenes, one launch per phase ----
 * The scenes are packed into one disjoint union, so per-tet, per-contact and
 * sparse-matrix work of all scenes runs in single launches; each scene keeps
 * its own Woodbury capacitance and its own GMRES (Sec. 5.4), and the Krylov
 * cycles of all scenes run in lockstep with a per-scene convergence mask.
 * Packed arrays: the vertices (and DOFs) of scene s occupy [voff[s],
 * voff[s+1]) in scene order (adj_batch_info). */
typedef struct adj_batch adj_batch; /* opaque */

/* descs: host [n_scenes], each as for adj_scene_create (the scenes must share
 * density, h and eps); max_contacts: host [n_scenes].  Errors as for
 * adj_scene_create. */
adj_status adj_batch_create(int32_t n_scenes, const adj_scene_desc* descs, const int32_t* max_contacts,
                            adj_batch** out);
adj_status adj_batch_destroy(adj_batch* batch);

/* out: host int64 [2 * (n_scenes + 1)]: vertex offsets, then tet offsets. */
adj_status adj_batch_info(const adj_batch* batch, int64_t* out);

/* Per-scene setup (a1-a4 for every scene): contacts: host [n_scenes] of
 * contact states (device arrays, vertex ids local to the scene, sorted; mu
 * per scene); q: device packed [n_verts_total * 3].  A scene may have at
 * most 8192 capacitance rows and 2730 contact vertices (ADJ_E_SHAPE). */
adj_status adj_batch_setup(adj_batch* batch, const adj_contact_state* contacts, const double* q,
                           const adj_solve_opts* opts, void* stream);

/* One GMRES per scene on Acal_s^T z_s = dL_dq_s + dL_dv_s / h to opts->rtol
 * (each scene's own right-hand side norm); ADJ_MIXED as for adjoint_solve.
 * dL_dq, dL_dv, z: device packed; info: host [n_scenes] or NULL.
 * ADJ_E_INVERTED / ADJ_E_SINGULAR when the last adj_batch_setup raised the
 * device error flag (an inverted tet or a singular capacitance pivot in any
 * scene), else ADJ_E_NOCONV if any scene did not converge (z holds the best
 * iterate). */
adj_status adj_batch_solve(adj_batch* batch, const double* dL_dq, const double* dL_dv, double* z,
                           const adj_solve_opts* opts, adj_solve_info* info, void* stream);

/* Gradient contractions of every scene (as vjp_params): packed vectors;
 * grad: device [n_scenes * 3] (dL/dE, dL/dnu, dL/dmu), accumulated (+=). */
adj_status adj_batch_vjp(adj_batch* batch, const double* z, const double* dL_dv, double* dL_dqbar,
                         double* dL_dvbar, double* dL_dfext, double* grad, void* stream);

/* Reverse pass over n_steps recorded steps of a batch (the time recursion of
 * Sec. 5.1): for t = n_steps-1 down to 0, setup at (q[t], contacts[t]),
 * one GMRES per scene on Acal_t^T z = gq + gv / h, the gradient contractions,
 * then gq <- dL/dqbar, gv <- dL/dvbar.  The setup of step t-1 needs no
 * gradient, so it runs on a second stream of the library's while step t is
 * solved: b0 and b1 are two batches created from the same scene
 * descriptions and take the steps in turn (step t on b0 when t is even).
 * contacts: host [n_steps][n_scenes] (device arrays as for adj_batch_setup);
 * q: host [n_steps] of device packed states; gq, gv: device packed, in: the
 * loss gradients w.r.t. the last state, out: w.r.t. the state before step
 * 0; dfext: host [n_steps] of device packed outputs (dL/df_ext of step t)
 * or NULL; grad: device [n_scenes * 3], accumulated over the steps; info:
 * host [n_steps][n_scenes] or NULL.  The call returns when the last solve
 * has been read back (the last contractions may still run on `stream`).
 * Errors as for the batch calls; ADJ_E_NOCONV (after finishing the pass)
 * if a scene did not converge in some step.  Device-side setup errors are
 * reported by adj_batch_check_status on either batch. */
adj_status adj_batch_reverse(adj_batch* b0, adj_batch* b1, int32_t n_steps, const adj_contact_state* contacts,
                             const double* const* q, double* gq, double* gv, double* const* dfext, double* grad,
                             const adj_solve_opts* opts, adj_solve_info* info, void* stream);

/* As adj_check_status, for the batch's last setup. */
adj_status adj_batch_check_status(adj_batch* batch, void* stream);

/* Diagnostics (synchronises the device): copy an array of one scene of the
 * last setup to host memory.  what = 0: Delassus matrix [n_cv][n_cv];
 * 1: capacitance inverse [mp][mp]; 2: Z = A^{-1} E [n_verts][n_cv]; 3: Y = S E
 * [n_verts][n_cv].  *size_bytes receives the size; ADJ_E_SHAPE when
 * capacity_bytes is smaller.  For tests and debugging. */
adj_status adj_batch_debug_export(const adj_batch* batch, int32_t what, int32_t scene, void* host_out,
                                  int64_t capacity_bytes, int64_t* size_bytes);

/* The union scene of the batch (owned by the batch; valid until
 * adj_batch_destroy), for adj_debug_export and adj_scene_info. */
adj_status adj_batch_scene(adj_batch* batch, adj_scene** out);

/* Launch shapes of the batched Krylov loop.  chunk: iterations enqueued
 * between host checks after the first chunk of a cycle (1..64; the first
 * runs as many as the last solve of the same kind needed); graph: 1 replays
 * each chunk from a HIP graph captured once per adj_batch_setup on the
 * batch's private stream (the same kernels, so results are bitwise those of
 * direct launches); a_inv: A^{-1} of the union in the preconditioner, 1 = the
 * sparse-inverse products S^T S, 2 = level-scheduled sweeps with the union's
 * Cholesky factor (every level one launch over all scenes), 0 = automatic
 * (sweeps when S holds more than 32 million and more than 4 nnz(L) entries).
 * Defaults: chunk 8, graph 0, a_inv 0.  ADJ_E_ARG outside these. */
typedef struct {
  int32_t chunk;
  int32_t graph;
  int32_t a_inv;
} adj_batch_tuning;
adj_status adj_batch_set_tuning(adj_batch* batch, const adj_batch_tuning* t);
adj_status adj_batch_get_tuning(const adj_batch* batch, adj_batch_tuning* t);

/* Batched autotuner (a9): after adj_batch_setup, times adj_batch_solve with
 * the right-hand side (dL_dq, dL_dv) for a_inv in {1, 2} (when the union has
 * the sweep structure), then chunk in {2, 4, 8, 16, 32} with direct
 * launches, then graph replay at the best chunk (each candidate the
 * best of `reps` timed solves, HIP events on `stream`, chunk graphs
 * re-captured for every solve as after a fresh setup), keeps the fastest on
 * the batch and writes it to *best.  z: device scratch [3 * total vertices]
 * that receives the last solution.  Synchronises the stream. */
adj_status adj_batch_autotune(adj_batch* batch, const double* dL_dq, const double* dL_dv, double* z,
                              const adj_solve_opts* opts, int32_t reps, adj_batch_tuning* best, void* stream);

const char* adj_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
