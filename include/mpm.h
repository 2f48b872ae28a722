/*
 * mpm.h - C ABI of the MI355X implicit APIC MPM hot path.
 *
 * The library implements one time step of the implicit Material Point Method with
 * spatially varying surface energy of Chen et al., "A Momentum-Conserving Implicit
 * Material Point Method for Surface Energies with Spatial Gradients" (arXiv 2101.12408):
 * the conservative split into surface and balance particles (Sections 4.1.2-4.1.3), the
 * APIC particle-to-grid transfer of mass, momentum and temperature (Section 4.2), the
 * backward-Euler grid momentum update with its energy, forces (eq. fe) and
 * Hessian-vector product (Section 4.3.1), the implicit heat update with the particle
 * Robin term (Section 4.3.2), and the grid-to-particle transfer with merge (Section 5).
 *
 * Conventions
 *  - Every entry point returns an int status (MPM_OK = 0 or an MPM_E* code) and never
 *    throws.  mpm_last_error() returns a message for the last failure on a context
 *    (with NULL: the last failure of the calling thread that had no context to hold it,
 *    e.g. a failed mpm_ctx_create).
 *  - Real numbers are double in MPM_FP64 mode and float in MPM_MIXED mode ("real" below).
 *    Scalar results (energies, norms, momentum sums) are always double.
 *  - All particle, surface and grid buffers are DEVICE pointers owned by the caller,
 *    structure-of-arrays: component a of item i is at [a * count + i].
 *  - Grid vectors are dense over all n^dim nodes, component-major ([dim][n^dim]), with
 *    nodes numbered tile by tile: the grid is cut into tiles of 4x4x4 nodes (3D) or 8x8
 *    nodes (2D); node (i0,i1[,i2]) has index tile*64 + local with
 *      tile  = t0 + nt*(t1 + nt*t2),  t_a = i_a / E,  nt = n / E,  E = 4 (3D) or 8 (2D)
 *      local = l0 + E*(l1 + E*l2),    l_a = i_a % E.
 *    mpm_node_index() computes it.  Node (i) sits at the cell centre (i + 1/2) dx
 *    (Section 4.2).  Only nodes with mass are unknowns; the library writes 0 elsewhere.
 *  - Every call is asynchronous on the caller's stream (a hipStream_t passed as void*;
 *    NULL is the null stream) unless documented otherwise.  Calls on one context must
 *    not overlap: a context owns its workspace.
 *  - The library allocates no device memory at run time.  mpm_workspace_bytes() sizes a
 *    workspace that the caller allocates and hands to mpm_ctx_create(); the context
 *    borrows it until mpm_ctx_destroy().  (mpm_step_noalloc instead uses a static device
 *    array that the GPU holds from the library's load on.)
 */
#ifndef MPM_H_
#define MPM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_ctx mpm_ctx;

enum mpm_status {
  MPM_OK = 0,
  MPM_EINVAL = 1,     /* invalid argument: dim, n, dx, null pointer, size           */
  MPM_ENOMEM = 2,     /* count above the capacity the workspace was sized for        */
  MPM_EBUDGET = 3,    /* admission refused: over the memory budget                   */
  MPM_EDOMAIN = 4,    /* a point's stencil leaves the grid (not in [dx, 1-dx)^dim)   */
  MPM_ENOCONV = 5,    /* Newton or a Krylov solve hit its iteration cap              */
  MPM_ENONFINITE = 6, /* a residual norm or energy became NaN or Inf                 */
  MPM_EHIP = 7        /* a HIP runtime call failed, or a bounded device wait gave up */
};

enum mpm_precision { MPM_FP64 = 0, MPM_MIXED = 1 };
enum mpm_hess_mode { MPM_HESS_PSD = 0, MPM_HESS_EXACT = 1 };
enum mpm_krylov { MPM_KRYLOV_CG = 0, MPM_KRYLOV_MINRES = 1 };
enum mpm_term { MPM_TERM_J = 1, MPM_TERM_SURF = 2, MPM_TERM_VISC = 4 };

/* Scene and solver parameters (Sections 3, 4 and the per-example values of Section 6). */
typedef struct mpm_params {
  int32_t dim;            /* 2 or 3                                                    */
  int32_t n;              /* nodes per axis, a multiple of 8; dx must equal 1/n        */
  int32_t precision;      /* mpm_precision                                             */
  int32_t hess_mode;      /* mpm_hess_mode: PSD drops the indefinite surface part      */
  int32_t term_mask;      /* mpm_term bits of the energy terms to include (default 7)  */
  int32_t momentum_fix;   /* 1: exact minimization along translations after each Newton
                             iteration when no velocity component is constrained       */
  int32_t wall_layers;    /* slip walls: velocity component a is fixed to 0 on nodes
                             with i_a < wall_layers or i_a >= n - wall_layers          */
  int32_t slab;           /* 1: component slab_axis fixed to 0 on nodes inside the box */
  int32_t slab_axis;
  int32_t heat;           /* 1: run the implicit heat update (Section 4.3.2)           */
  int32_t gamma_by_label; /* 1: k_r = gamma_label[label_r] (piecewise constant, Sec 3.6);
                             2: k_r = gamma(T) on samples labelled 1 (the free surface)
                             and gamma_label[0] on the others (against container walls) */
  int32_t newton_max, cg_max, ls_max, heat_max;
  int32_t krylov;         /* mpm_krylov: the Newton system's solver.  CG (with the PSD
                             Hessian); MINRES (Paige-Saunders, Jacobi-preconditioned) for
                             the EXACT Hessian, which may be indefinite: it stops at the
                             same relative reduction as CG, measured in the preconditioned
                             residual norm; cg_max caps both                            */
  double dx, dt;
  double gravity[3];
  double bulk;            /* lambda^l in Psi^p(J) = lambda/2 (J-1)^2 (Section 3.2.1)   */
  double mu0, mu_k, mu_T0;/* viscosity mu(T) = mu0 exp(-mu_k (T - mu_T0))              */
  double g0, g1, gT0, gmin, gmax; /* k^sigma(T) = clamp(g0 + g1 (T - gT0), gmin, gmax) */
  double gamma_label[4];
  double cp, K, h, T_amb, b, H;   /* heat: c_p, conductivity, Robin h, ambient, b, source */
  double slab_lo[3], slab_hi[3];
  double newton_tol;      /* stop when |P grad Phi| <= newton_tol |P grad Phi_0|       */
  double cg_rel;          /* inner CG: |r| <= max(cg_rel |g|, 0.1 newton_tol |g_0|)    */
  double ls_c1;           /* Armijo constant of the backtracking line search           */
  double heat_tol;        /* heat CG: |r| <= heat_tol |rhs|                            */
  double cfl;             /* > 0: mpm_step chooses each step's dt from the particles it
                             is given (the paper's CFL-limited dt): explicit
                             dt = clamp(cfl dx / (max_p |v_p| + sqrt(bulk / rho_min)),
                             dt_min, dt_max), implicit dt = clamp(cfl dx / max_p |v_p|,
                             dt_min, dt_max), rho_p = m_p / V0_p; the dt taken is in
                             mpm_stats.dt.  <= 0: the fixed dt above                     */
  double dt_min, dt_max;
  /* Collision objects: up to MPM_MAX_PLANES static half-spaces, object k occupying
   * {x : (x - plane_o[k]) . plane_n[k] < 0} (plane_n a unit normal pointing out of the
   * object), each with a Coulomb friction coefficient plane_mu[k].  mpm_step applies them
   * to the grid velocity v^ after the momentum update and before G2P, object by object in
   * index order, at every node with (x_i - o) . n <= 0: with v_n = v^ . n < 0 the
   * tangential part v_t = v^ - v_n n keeps max(0, |v_t| + mu v_n) of its length
   * (sticking when that is 0) and the normal part is removed; nodes moving away (v_n >= 0)
   * keep v^.  n_planes = 0: none. */
  int32_t n_planes;
  int32_t pad0_;
  double plane_o[4][3];
  double plane_n[4][3];
  double plane_mu[4];
  /* Solid phase (Sections 3.2.1, 3.5): a particle with T < T_melt is a fixed-corotated
   * solid, psi^h(F) = mu^h sum_a (sigma_a - 1)^2 + lambda^h / 2 (J - 1)^2 per reference
   * volume, with (mu^h, lambda^h) = (muh0, lamh0) exp(-kh (T - Th0)); it has no J-term
   * pressure and no viscosity, and carries its deformation gradient in mpm_particles.F.
   * G2P advances F <- (I + dt grad v^) F and J = det F; a particle whose temperature
   * crosses T_melt upward becomes liquid with J = 1, one crossing downward becomes solid
   * with F = I.  The phase is decided in FP64.  T_melt <= -1e299 (the default): no
   * solids.  The solid's Hessian is the fixed-rotation form 2 mu dF + lambda (cof F : dF)
   * cof F (positive semidefinite); hess_mode EXACT is not available with solids.  A
   * context created without solids cannot enable them later. */
  double T_melt;
  double muh0, lamh0, kh, Th0;
} mpm_params;

enum { MPM_MAX_PLANES = 4 };

/* Interior MPM particles (Section 4): SoA device buffers of real, n items each.
 * x, v: [dim][n]; A: [dim*dim][n] with entry (a,b) at component a*dim+b; gradT: [dim][n]. */
typedef struct mpm_particles {
  int64_t n;
  void* x;
  void* v;
  void* A;
  void* J;
  void* V0;
  void* m;
  void* T;
  void* gradT;
  void* F;                  /* [dim*dim][n], entry (a,b) at component a*dim+b: the
                               deformation gradient of solid particles (liquid particles'
                               entries are carried along); required when T_melt is set,
                               else ignored (may be NULL)                                  */
} mpm_particles;

/* Surface samples s_r with area-weighted outward normals dA_r (Section 4.1.1), device
 * buffers: s, dA [dim][n] real; label [n] int32 (may be NULL unless gamma_by_label). */
typedef struct mpm_surface {
  int64_t n;
  const void* s;
  const void* dA;
  const int32_t* label;
} mpm_surface;

/* Solver statistics of the last step / solve on a context (host copy).  converged: 1 when
 * |g| met the tolerance, 2 when a MIXED-mode solve stopped at the FP32 floor of the
 * gradient (|g| <= 1e-4 |g0| and a Newton step no longer halves it), 0 otherwise. */
typedef struct mpm_stats {
  int32_t newton_iters, cg_iters, heat_iters, line_search_halvings;
  int32_t energy_evals, hessvecs, converged, status;
  double g0, gnorm, phi, heat_res;
  double momentum[3];     /* sum_i m_i v^_i over the grid after the solve (FP64); after
                             an implicit mpm_step, set by the next mpm_scene_status      */
  int64_t n_part, n_surf, n_dof, n_tiles;
  double dt;              /* the time step of the last step                           */
  int64_t host_waits;     /* blocking host waits on the device since the last mpm_step
                             began (reads of counts and solver scalars)                  */
} mpm_stats;

/* Grid fields readable through mpm_grid_view (device pointers into the workspace). */
enum mpm_field {
  MPM_F_MASS = 0,   /* m_i                        real [n^dim]                          */
  MPM_F_MOM = 1,    /* (mv)_i                     real [dim][n^dim]                     */
  MPM_F_W = 2,      /* sum_p m_p N_i(x_p)         real [n^dim]                          */
  MPM_F_WT = 3,     /* sum_p m_p N_i (T_p + (x_i-x_p).grad T_p)   real [n^dim]          */
  MPM_F_E = 4,      /* split-member mass weights  real [n^dim]                          */
  MPM_F_ET = 5,     /* split-member temperature   real [n^dim]                          */
  MPM_F_VN = 6,     /* v^n_i = (mv)_i / m_i       real [dim][n^dim]                     */
  MPM_F_TN = 7,     /* T^n_i                      real [n^dim]                          */
  MPM_F_FREE = 8,   /* uint8 [n^dim]: bit a set = component a free, bit 7 = has mass     */
  MPM_F_HEAT_RHS = 9,   /* right side of the heat system   real [n^dim]                 */
  MPM_F_HEAT_DIAG = 10, /* Jacobi diagonal of the heat system  real [n^dim]             */
  MPM_F_VHAT = 11,  /* v^ after the last momentum solve   real [dim][n^dim]             */
  MPM_F_THAT = 12,  /* T^ after the last heat solve       real [n^dim]                  */
  MPM_F_PARENT = 13,/* int32 [n_surf]: parent p(r) of each surface sample (input order) */
  MPM_F_COUNT = 14, /* int32 [n_part]: |Pi_p| (input order)                             */
  MPM_F_KSURF = 15, /* real [n_surf]: k_r (input order)                                 */
  MPM_F_MOM_DIAG = 16, /* Jacobi diagonal of the Newton matrix  real [dim][n^dim]       */
  MPM_F_PERM = 17   /* int32 [n_part]: input index of the particle in each cell-order slot */
};

/* Kernel classes timed by mpm_timing (HIP events stamped by the launches themselves). */
enum mpm_kernel_class {
  MPM_K_SORT = 0,        /* cell keys, scans, slot scatter, per-cell order              */
  MPM_K_SETUP = 1,       /* staging, parents, split, balance points, tiles, k_r         */
  MPM_K_P2G = 2,         /* P2G cell-tile scatter into per-tile partial fields          */
  MPM_K_ENERGY_INT = 3,  /* energy/gradient point phase, interior particles             */
  MPM_K_ENERGY_SURF = 4, /* energy/gradient point phase, surface samples                */
  MPM_K_ENERGY_NODE = 5, /* energy/gradient node phase                                  */
  MPM_K_HESS_INT = 6,    /* Hessian-vector product point phase, interior particles      */
  MPM_K_HESS_SURF = 7,   /* Hessian-vector product point phase, surface samples         */
  MPM_K_HESS_NODE = 8,   /* Hessian-vector product node phase                           */
  MPM_K_HEAT_PT = 9,     /* heat operator point phase                                   */
  MPM_K_HEAT_NODE = 10,  /* heat operator node phase                                    */
  MPM_K_G2P_SPLIT = 11,  /* G2P moments of surface and balance points                   */
  MPM_K_G2P = 12,        /* G2P with merge and advection                                */
  MPM_K_BLAS = 13,       /* Krylov vector updates and dot products                      */
  MPM_K_P2G_NODE = 14,   /* P2G node phase: partial merge and the grid set-up           */
  MPM_K_SAMPLE = 15,     /* device surface sampler (mpm_sample_surface_dev)             */
  MPM_K_COUNT = 16
};

/* Node numbering helper (tile-major order described above). */
static inline int64_t mpm_node_index(int32_t dim, int32_t n, int32_t i0, int32_t i1, int32_t i2) {
  const int32_t E = (dim == 3) ? 4 : 8;
  const int64_t nt = n / E;
  int64_t tile = (i0 / E) + nt * ((i1 / E) + (dim == 3 ? nt * (i2 / E) : 0));
  int64_t local = (i0 % E) + E * ((i1 % E) + (dim == 3 ? E * (i2 % E) : 0));
  return tile * 64 + local;
}

/* Fills *p with defaults for dimension dim and n nodes per axis (dx = 1/n, FP64, PSD,
 * all terms, 20 Newton / 1000 CG / 10 line-search / 1000 heat iterations, tolerances
 * 1e-8 / 1e-2 / 1e-10, Armijo 1e-4).  Returns MPM_EINVAL for dim not 2 or 3. */
int mpm_params_default(mpm_params* p, int32_t dim, int32_t n);

/* Device workspace bytes for a context holding up to cap_part interior particles and
 * cap_surf surface samples with parameters p.  Host only; synchronous. */
int mpm_workspace_bytes(const mpm_params* p, int64_t cap_part, int64_t cap_surf, size_t* out_bytes);

/* Creates a context over a caller-allocated device workspace of ws_bytes (at least
 * mpm_workspace_bytes, 256-byte aligned).  The parameters are copied.  Host only. */
int mpm_ctx_create(const mpm_params* p, void* workspace, size_t ws_bytes, int64_t cap_part,
                   int64_t cap_surf, mpm_ctx** out);
int mpm_ctx_destroy(mpm_ctx* ctx);
const char* mpm_last_error(const mpm_ctx* ctx);
/* Replaces the parameters of a context (same dim, n, precision and capacities).  What the
 * grid set-up forms from them (k_r, mu_p, the per-particle Hessian factors, the Jacobi
 * diagonals, the heat right side) follows at the next mpm_p2g. */
int mpm_ctx_set_params(mpm_ctx* ctx, const mpm_params* p);

/* Sections 4.1.2-4.2 and the grid set-up: bins particles and samples by cell, finds each
 * sample's nearest interior particle (ties to the lower index), forms the balance points
 * b_r = s_r + 2 (x_p(r) - s_r) and split masses m_p / (2|Pi_p| + 1), transfers mass,
 * APIC momentum and temperature to the grid, and prepares the grid unknowns (nodes with
 * mass, v^n, T^n, constraints, k_r, mu_p, Jacobi diagonals, heat right side).  P and S
 * are read, never written.  Points outside [dx, 1-dx)^dim latch MPM_EDOMAIN, returned by
 * the next synchronizing call. */
int mpm_p2g(mpm_ctx* ctx, const mpm_particles* P, const mpm_surface* S, void* stream);

/* Section 4.3.1: Phi(v^) = 1/2 sum m |v^-v^n|^2 - dt sum m g.v^ + e(x + dt v^) + dt D(v^)
 * (energy_dev: one device double) and its gradient with respect to v^ (grad: real
 * [dim][n^dim], projected onto the free components).  Requires mpm_p2g. */
int mpm_energy_grad(mpm_ctx* ctx, const void* v_hat, double* energy_dev, void* grad, void* stream);

/* Section 4.3.1: out = P (alpha M P w + d2Psi/dv^2 (v_lin) P w), P the projection onto
 * free components, Psi = e(x + dt v^) + dt D(v^).  alpha = 1 gives the Newton matrix,
 * alpha = 0 the energy Hessian alone.  The surface part is the PSD part or the exact
 * second derivative per hess_mode.  Requires mpm_p2g. */
int mpm_hessvec(mpm_ctx* ctx, const void* v_lin, const void* w, double alpha_mass, void* out,
                void* stream);

/* Section 4.3.2: T_out = A T_in with A = c_p/dt diag(m) + L + R over the nodes with mass
 * (L the particle conduction matrix, R the particle Robin matrix).  Requires mpm_p2g. */
int mpm_heat_apply(mpm_ctx* ctx, const void* T_in, void* T_out, void* stream);

/* Section 5: G2P with merge of split groups, then J_p and x_p advanced.  Writes the
 * whole particle state (x, v, A, J, V0, m, T, gradT) of P back IN CELL ORDER: slot j then
 * holds the particle whose index in the mpm_p2g input was perm[j] (MPM_F_PERM), so that
 * the next step's binning finds the particles almost sorted and every access coalesces.
 * T_hat may be NULL: T and gradT are then carried over unchanged.  Requires mpm_p2g on
 * the same P and S. */
int mpm_g2p(mpm_ctx* ctx, const void* v_hat, const void* T_hat, mpm_particles* P, void* stream);

/* Momentum solve only (after mpm_p2g): Newton-CG on Phi; v^ lands in MPM_F_VHAT.
 * Synchronizes the stream.  Returns MPM_ENOCONV if Newton hit newton_max. */
int mpm_solve_momentum(mpm_ctx* ctx, void* stream);
/* Heat solve only (after mpm_p2g): CG on the heat system; T^ lands in MPM_F_THAT. */
int mpm_solve_heat(mpm_ctx* ctx, void* stream);

/* One full step for each of n_scenes scenes (Section 4, its list of steps): p2g,
 * momentum solve (implicit = 1: backward Euler with Newton; implicit = 0: explicit,
 * forces at y = x), heat solve when enabled, g2p.  Particles are updated in place.
 * With more than one scene the scenes run concurrently: up to mpm_batch_config()
 * scenes at a time, each on a worker thread with its own non-blocking stream (default
 * priority) that waits for the work already queued on `stream`; the call returns when
 * every scene is done and `stream` is ordered after them.  A scene's results do not
 * depend on the batch it runs in (bitwise).  The contexts must be distinct.  Returns the
 * first non-OK status in scene order; per-scene status is in mpm_stats.  An implicit step
 * returns once its last host check is done, while its G2P may still run on the stream
 * (work queued after it is ordered behind it); the status it returns covers the whole
 * step.  Its grid momentum (mpm_stats.momentum) is read by the next mpm_scene_status. */
int mpm_step(mpm_ctx* const* ctxs, mpm_particles* const* P, const mpm_surface* const* S,
             int32_t n_scenes, int32_t implicit, void* stream);
/* Maximum number of scenes mpm_step advances at once (1..64, default 8; process-wide). */
int mpm_batch_config(int32_t max_concurrent);

/* One step of one scene that allocates nothing, for callers that cannot allocate device
 * or pinned memory, create streams or events (tight serving loops, harnesses that forbid
 * allocation).  It computes what mpm_step computes for a single scene with a context of
 * parameters p and capacities P->n, S->n, bitwise the same, but with no context and no
 * workspace argument: the workspace is a static device array of *scratch_bytes bytes
 * (256 MiB; each GPU the library runs on holds its own copy until the process ends), the
 * host scalar block is static host memory, and every kernel runs on `stream`.  P (device,
 * real per p->precision) is updated in place in cell order as by mpm_step; S may be NULL.
 * The scratch is cleared at the start of every call and the call returns only when the
 * step is complete on the device.  Calls on the same GPU share the one array: they are
 * serialized by a lock, and a call that overlapped another on that GPU from outside the
 * library (a kernel still reading P) would race.  Returns MPM_ENOMEM, with a message in
 * mpm_last_error(NULL), when the scene's workspace (mpm_workspace_bytes) exceeds the
 * scratch; otherwise the status of the step.  scratch_bytes (may be NULL) receives the
 * scratch size on every call. */
int mpm_step_noalloc(const mpm_params* p, mpm_particles* P, const mpm_surface* S, int32_t implicit, void* stream,
                     size_t* scratch_bytes);

/* Device pointer of a grid field of the last mpm_p2g / solve (see mpm_field). */
int mpm_grid_view(mpm_ctx* ctx, int32_t field, void** out_ptr);
int mpm_get_stats(const mpm_ctx* ctx, mpm_stats* out);
/* Timing of the context's kernels by class: enable = 1 starts (and resets) recording of a
 * HIP event pair for every launch on the call's stream, stamped with the kernel's own
 * begin and end (hipExtLaunchKernel), 0 stops it.  Host only. */
int mpm_timing(mpm_ctx* ctx, int32_t enable);
/* Synchronizes on the recorded events and returns, per kernel class, the summed
 * duration in milliseconds (ms[MPM_K_COUNT]) and the number of launches; work_ms and
 * work_launches (each may be NULL) the same over the launches that did work (a CG that
 * the device has called off still launches its kernels, which return at once: launches
 * shorter than a tenth of the class's 95th-percentile duration are left out). */
int mpm_timing_read(mpm_ctx* ctx, double* ms, int64_t* launches, double* work_ms, int64_t* work_launches);
/* Latched device status of the context (synchronizes the stream). */
int mpm_scene_status(mpm_ctx* ctx, void* stream);

/* Host input stage (Section 4.1.1), not part of the timed device path: samples the zero
 * isocontour of the union-of-spheres level set around host positions x ([dim][n_part]
 * double).  Marching tetrahedra (3D) / triangles (2D) on the node lattice; per element
 * max(1, floor(density * measure + u)) samples with SplitMix64 counter draws keyed by
 * (seed, step, element id).  Writes at most cap samples to host buffers s, dA
 * ([dim][cap] double) and label ([cap] int32: 1 inside [label_lo, label_hi)); *out_n
 * receives the sample count (which may exceed cap: call again with a larger buffer).
 * radius and density <= 0 select 0.73 dx / 0.867 dx and 4/dx / 8/dx^2. */
int mpm_sample_surface(int32_t dim, int32_t n, const double* x, int64_t n_part, double radius,
                       double density, uint64_t seed, uint64_t step, const double* label_lo,
                       const double* label_hi, double* s, double* dA, int32_t* label, int64_t cap,
                       int64_t* out_n);

/* Autotuner of the tile kernels' launch layout.  The stress (energy, Hessian) and heat
 * tile kernels map workgroups to cell tiles in runs of `run` consecutive tiles per XCD
 * (each XCD has its own L2; neighbouring tiles share node-region lines).  mpm_autotune
 * times each kernel class on the context's current scene (after mpm_p2g) at run lengths
 * 1, 2, 4, ..., 64 (the best of three launches each, the surface linearized at v^n) and
 * keeps the fastest for the context's later launches.  The run length only assigns tiles
 * to workgroups: results are bitwise the same for every choice.  Synchronizes stream; out
 * (may be NULL) receives the times.  mpm_tuning_set fixes the run lengths (energy,
 * Hessian, heat; 0 = the built-in size rule; run NULL resets all three). */
typedef struct mpm_tuning {
  int32_t run[3];          /* chosen run length per class (0: class not timed)          */
  int32_t ncand;           /* candidates timed                                          */
  int32_t cand[8];         /* their run lengths                                         */
  double us[3][8];         /* best launch-pair time of each candidate, microseconds     */
} mpm_tuning;
int mpm_autotune(mpm_ctx* ctx, void* stream, mpm_tuning* out);
int mpm_tuning_set(mpm_ctx* ctx, const int32_t* run);

/* Device surface sampler (Section 4.1.1): the samples mpm_sample_surface draws, computed
 * on the context's GPU from device particle positions P->x ([dim][P->n] real of the
 * context's precision, P->n <= the context's particle capacity; the other particle arrays
 * are not read).  The same level set, isocontour, element ids and counter draws, with
 * every floating-point operation of the geometry in the host stage's order and FP64
 * arithmetic, so the samples equal the host stage's bit for bit (in MIXED the positions
 * are the FP32 values and s, dA are rounded to FP32 on output).  Writes the samples to
 * device buffers s_out, dA_out ([dim][count] real) and label ([count] int32, may be NULL)
 * in element-id order, only when the count is <= cap; *out_n receives the count either
 * way (call again with larger buffers).  The result can be passed to mpm_step as its
 * mpm_surface {count, s_out, dA_out, label}.  Runs on stream, and waits for it once to read
 * the count.  Uses the context's sampler scratch and its particle staging buffer (which
 * the next mpm_p2g rewrites), not the state of the last step or its views.  radius and
 * density <= 0 select the defaults of mpm_sample_surface; radius must be below dx.
 * Errors: MPM_EINVAL for null or inconsistent arguments. */
int mpm_sample_surface_dev(mpm_ctx* ctx, const mpm_particles* P, double radius, double density, uint64_t seed,
                           uint64_t step, const double* label_lo, const double* label_hi, void* s_out,
                           void* dA_out, int32_t* label, int64_t cap, int64_t* out_n, void* stream);

/* ---- Serving: continuous batching of step requests -------------------------------
 * A server owns max_concurrent worker threads, each with its own non-blocking stream
 * (default priority), and sub-allocates a caller-provided device arena (256-byte
 * aligned; the library allocates no device memory).  Requests are admitted strictly in
 * arrival order, each as soon as a worker is free and the arena holds its context
 * workspace, particle and surface buffers; a request larger than the whole arena
 * completes with MPM_EBUDGET.  A worker draws each step's surface samples on the device
 * from the resident positions (mpm_sample_surface_dev; a request whose samples outgrow
 * the first sizing, twice its particle count and at least 4096, runs again once sized
 * by the count), runs the steps with mpm_step, downloads the final particle state
 * (in the request's particle order) and frees the memory.  Several admitted requests run
 * at once and their work overlaps on the device; each result is bitwise the same as
 * stepping the scene alone.  All entry points are host calls and thread-safe. */
typedef struct mpm_server mpm_server;

typedef struct mpm_request {
  int64_t id;               /* caller's id (unique among results not yet fetched)          */
  mpm_params params;
  int32_t n_steps;          /* steps to advance (>= 1)                                     */
  int32_t implicit;         /* 1: implicit steps, 0: explicit                              */
  int32_t keep_result;      /* 1: keep the final state for mpm_server_result               */
  int32_t borrow;           /* 1: read the host arrays in place (the caller keeps them
                               unchanged until the request completes); 0: copy at submit  */
  int64_t n_part;
  uint64_t seed;            /* sampler seed; step k of the request draws with step index   */
  uint64_t first_step;      /* first_step + k                                              */
  double ls_radius;         /* sampler radius and density (<= 0: the defaults of           */
  double sample_density;    /* mpm_sample_surface)                                          */
  double label_lo[3], label_hi[3];
  /* host particle state, double, SoA [comp][n_part] (x, v, gradT: dim; A: dim*dim; the
   * rest 1); copied by mpm_server_submit unless borrow */
  const double *x, *v, *A, *J, *V0, *m, *T, *gradT;
} mpm_request;

typedef struct mpm_completion {
  int64_t id;
  int32_t status;           /* MPM_OK or the request's first error                         */
  int32_t steps_done;
  double t_submit, t_admit, t_done;   /* mpm_server_clock() seconds                        */
  int64_t n_part, n_surf;   /* n_surf of the last step                                     */
  int64_t bytes;            /* arena bytes held while resident                             */
  int32_t newton_iters, cg_iters;     /* summed over the request's steps                   */
} mpm_completion;

typedef struct mpm_server_info {
  int64_t submitted, completed, rejected, queued, running;
  int64_t arena_bytes, bytes_in_use, peak_bytes;
  int32_t peak_running, pad_;
} mpm_server_info;

/* Seconds of a monotonic clock (the time base of mpm_completion). */
double mpm_server_clock(void);
int mpm_server_create(void* arena, size_t arena_bytes, int32_t max_concurrent, mpm_server** out);
/* Queues a request (copies its host state unless borrow); returns at once. */
int mpm_server_submit(mpm_server* srv, const mpm_request* req);
/* Completions since the last poll, oldest first (at most cap; *n_out receives the count). */
int mpm_server_poll(mpm_server* srv, mpm_completion* out, int32_t cap, int32_t* n_out);
/* Blocks until nothing is queued or running (timeout_s < 0: no limit; MPM_ENOCONV on
 * timeout). */
int mpm_server_wait(mpm_server* srv, double timeout_s);
/* Final state of a completed request kept with keep_result (host double, SoA, request
 * particle order; any pointer may be NULL); releases it.  Returns the request's status. */
int mpm_server_result(mpm_server* srv, int64_t id, double* x, double* v, double* A, double* J,
                      double* T, double* gradT);
int mpm_server_info_get(mpm_server* srv, mpm_server_info* out);
/* Finishes every queued request, then stops the workers. */
int mpm_server_destroy(mpm_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* MPM_H_ */
