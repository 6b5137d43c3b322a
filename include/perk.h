/* perk.h - C ABI of the MI355X partitioned P-ERK + DGSEM library (libperk.so).
 *
 * The library advances a method-of-lines system U' = F(U) obtained from a discontinuous
 * Galerkin spectral element discretisation (DGSEM, flux differencing on Legendre-Gauss-Lobatto
 * nodes) of the compressible Euler or Navier-Stokes (BR1) equations on a periodic Cartesian
 * forest of quad/octrees with 2:1 mortars, with a partitioned Paired-Explicit Runge-Kutta
 * (P-ERK) method whose members are assigned to the elements by their refinement level.
 *
 * Paper passages defining the operations (D. Doehring et al., "Multirate time-integration
 * based on dynamic ODE partitioning through adaptively refined meshes for compressible fluid
 * dynamics"):
 *   - partitioned system and partitioned RK step: Sec. 2, eq. (PartitionedODESys) and
 *     eq. (PartitionedRKSystem);
 *   - P-ERK tableaux (shared c and b, two nonzeros per row, internal consistency): Sec. 3.1,
 *     eq. (PERK_ButcherTableauClassic), Sec. 3.3, eq. (PERK_ThirdOrderShuOsher);
 *   - order conditions, internal consistency, conservation: eqs. (PRKOrderCondsSimplified),
 *     (InternalConsistency), (Conservation);
 *   - level-wise evaluation of the right-hand side over the elements of a partition and the
 *     assignment of elements, interfaces and mortars to partitions after every mesh change:
 *     Sec. 6.1, 6.2;
 *   - level -> method map when there are more levels than methods: Sec. 6.4.1 (Actual Number of
 *     Right-Hand-Side Evaluations);
 *   - scalar RHS-evaluation count: eq. (ActualRHSEvals).
 *
 * Conventions
 *   - Every call returns a pe_status; on failure pe_last_error(ctx) describes it.  No call
 *     aborts or throws across the ABI.  Calls made in the wrong order return PE_ESTATE.
 *   - Device pointers are HIP device addresses on the current device; host pointers are
 *     ordinary memory.  The caller owns every buffer it passes; the library never frees them.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls that take a stream are
 *     asynchronous on it unless stated otherwise.
 *   - One context per host thread.  Calls on one context must not overlap.
 *   - All floating point is fp64.
 *
 * State layouts
 *   - "leaf layout" (what the caller sees): [leaf][var][node], leaves in the order of the
 *     leaf list given to pe_mesh_build, vars = rho, rho v_1 .. rho v_d, E, node index
 *     i + N j (+ N^2 k) with N = degree + 1.
 *   - "slot layout" (what the library steps): [var][slot][node], slots = elements sorted by
 *     partition, finest partition first, leaf order inside a partition.  The elements active
 *     at any stage form a prefix of the slots.  pe_element_info maps slots to leaves.
 */
#ifndef PERK_H
#define PERK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pe_ctx pe_ctx;
typedef struct pe_batch pe_batch;

typedef enum {
  PE_OK = 0,
  PE_EINVAL = -1,        /* invalid argument (shape, range, unbalanced mesh, bad tableau) */
  PE_ENOMEM = -2,        /* host allocation failed */
  PE_EHIP = -3,          /* a HIP runtime call failed */
  PE_ESTATE = -4,        /* call out of order (e.g. step before partition or bind) */
  PE_ENONFINITE = -5,    /* non-finite or non-positive density/pressure detected */
  PE_EUNSUPPORTED = -6   /* valid but not built (dimension / degree / equations combination) */
} pe_status;

typedef struct {
  int dim;          /* 2 or 3 */
  int degree;       /* polynomial degree k; built: 2 and 3 (N = k+1 LGL nodes per direction) */
  int equations;    /* 0: compressible Euler; 1: compressible Navier-Stokes with BR1 */
  double gamma;     /* ratio of specific heats */
  double mu;        /* dynamic viscosity (Navier-Stokes only, constant) */
  double prandtl;   /* Prandtl number (Navier-Stokes only); gas constant 1 */
} pe_physics;

typedef struct {
  int dim;
  int n_root[3];            /* trees per direction (third ignored in 2D) */
  double lo[3], hi[3];      /* box corners */
  int n_leaves;
  const int32_t* leaves;    /* host, [n_leaves][4]: (level, i, j, k); cell (i, j, k) of the uniform
                               grid with n_root[d] << level cells per direction; periodic box */
} pe_mesh_desc;

typedef struct {
  int order;                /* 2 or 3 (linear order of consistency p) */
  int n_members;            /* R, 1 <= R <= 8 */
  int n_stages;             /* S = E[R-1] (the largest member uses every stage), S <= 32 */
  const int32_t* E;         /* host [R]: stage evaluations per member, strictly ascending */
  const double* c;          /* host [S]: shared abscissae */
  const double* a_sub;      /* host [R][S]: per member and 0-based row i the one coefficient
                               beside the first column: a_{i,i-1} (classic pattern) or a_{i,j}
                               with j = coupling[r][i]; rows 0 and 1 are 0; a_{i,1} = c_i - a_sub
                               (internal consistency) */
  const double* b;          /* host [S]: shared weights */
  const int32_t* coupling;  /* host [R][S] or NULL.  NULL: the classic pattern of Sec. 3.1 (member
                               r evaluates stages 1 and S-E_r+2 .. S, row i couples K_{i-1}).
                               Otherwise an alternative stage-evaluation pattern (Sec. 3.2.4,
                               eq. PERK_ButcherTableauAlternating and eq.
                               PERK_ButcherTableauEarlyShared): the 0-based column j, 1 <= j < i, of
                               row i's coupling, or -1 for a row that is U_n + dt c_i K_1.  Each
                               K_j may feed at most one row per member; member r evaluates stage 1,
                               the stages with b != 0 and the coupled ones, E_r in number, and the
                               largest member all S.  The active elements of a stage are then a
                               union of member ranges rather than a prefix.  Euler only; no adjoint
                               and no batched runs with such patterns (PE_EUNSUPPORTED). */
} pe_perk_coeffs;

/* Create a context for the given physics.  No device work.  (Sec. 2, eq. ConservationLaw.) */
pe_status pe_create(pe_ctx** out, const pe_physics* phys);

/* Destroy a context.  Does not touch caller-owned device memory. */
void pe_destroy(pe_ctx* ctx);

/* Text of the last error on this context (valid until the next call on it). */
const char* pe_last_error(const pe_ctx* ctx);

/* Build the forest from a leaf list: periodic neighbour search, conforming faces and 2:1
 * mortars (Sec. 6.2).  Host only.  PE_EINVAL if the leaves overlap, leave holes or violate
 * 2:1 balance across faces.  Invalidates any binding: query sizes and bind again. */
pe_status pe_mesh_build(pe_ctx* ctx, const pe_mesh_desc* mesh);

/* Set the P-ERK family (Sec. 3.1, 3.3).  Checks to 1e-12: sum b = 1; b^T c = 1/2 (order >= 2);
 * b^T c^2 = 1/3 and b^T A^(r) c = 1/6 for every member (order 3), eq. (PRKOrderCondsSimplified);
 * the zero pattern a_{i,i-1}^(r) = 0 for i < S - E^(r) + 2 (0-based) so that member r evaluates
 * exactly stages 1 and S-E^(r)+2..S; every stage with b_i != 0 evaluated by every member.
 * Returns PE_EINVAL on violation; PE_EUNSUPPORTED for a coupling table on a Navier-Stokes
 * context or while shock capturing is on.  Invalidates the partition. */
pe_status pe_set_perk_coefficients(pe_ctx* ctx, const pe_perk_coeffs* coeffs);

/* Level -> member rules (which member of the family integrates the elements of each refinement
 * level; pe_partition and pe_amr_cycle apply the context's rule when they are given no map).
 *   PE_LEVEL_RULE_PAPER (the default; Sec. 6.4.1): the finest level takes the member with the most
 *     stage evaluations (R-1), the next coarser level R-2, and so on; every level beyond the R
 *     finest takes member 0 (the fewest evaluations).
 *   PE_LEVEL_RULE_REQUIRED_STEP: the spectrum of a convection-dominated discretisation scales with
 *     1/h (Sec. 3.1), so a member whose optimal step at the finest element size is dt_opt[r]
 *     admits dt_opt[r] 2^(finest - l) on level l.  Level l takes the cheapest member r that admits
 *     dt_opt[R-1] * margin (the common step set by the finest level, times a safety margin); the
 *     finest level takes member R-1; a level no member admits takes member R-1.  With margin 1
 *     and dt_opt doubling from member to member it gives the paper rule.
 * Levels finer than the finest level take member R-1 under both rules. */
typedef enum { PE_LEVEL_RULE_PAPER = 0, PE_LEVEL_RULE_REQUIRED_STEP = 1 } pe_level_rule;

/* Select the level rule of the context.  dt_opt (host [R], positive; ignored by the paper rule)
 * holds each member's optimal step at one common element size, margin >= 1.  The required-step
 * rule needs the coefficients set first (dt_opt has one entry per member); a later
 * pe_set_perk_coefficients with another member count clears it (PE_ESTATE until set again).
 * PE_EINVAL for an unknown rule, a non-positive or non-finite dt_opt entry or margin < 1. */
pe_status pe_set_level_rule(pe_ctx* ctx, int rule, const double* dt_opt, double margin);

/* The context's rule as a map: member_of_level[l] (host [n_levels], 1 <= n_levels <= 16) for a
 * mesh whose finest level is finest_level, or the finest level of the current mesh when
 * finest_level < 0.  Host only. */
pe_status pe_level_map(const pe_ctx* ctx, int finest_level, int n_levels, int32_t* member_of_level);

/* Sizes for the caller's allocations: the state (doubles, slot layout) and the workspace
 * (bytes, 256-byte aligned start required).  Valid after pe_mesh_build and
 * pe_set_perk_coefficients. */
pe_status pe_query_sizes(const pe_ctx* ctx, int64_t* n_state_doubles, int64_t* n_workspace_bytes,
                         int64_t* n_elements);

/* Reserve room for up to max_elements elements (default: the current element count) so that
 * adaptive meshes keep their buffers: the slot layout then has leading dimension max_elements.
 * Invalidates any binding: query sizes and bind again. */
pe_status pe_reserve(pe_ctx* ctx, int64_t max_elements);

/* Bind caller-owned device buffers of the sizes from pe_query_sizes and upload the mesh
 * tables into the workspace on `stream`.  The state content is undefined until
 * pe_set_state. */
pe_status pe_bind(pe_ctx* ctx, double* u_dev, void* workspace_dev, void* stream);

/* Re-flag elements into partitions on the device (Sec. 6.2): member of every element from
 * member_of_level (host, [n_levels] where n_levels = max leaf level + 1, values in [0, R)), or,
 * when member_of_level is NULL (n_levels ignored), from the context's level rule at the finest
 * level of the current mesh (pe_set_level_rule; by default the paper rule of Sec. 6.4.1),
 * stable counting sort of the elements by member (most stage evaluations first), remap of the
 * connectivity to the new slots, permutation of the bound state, per-stage active prefix
 * lengths.  Synchronises `stream` once to read the member counts back. */
pe_status pe_partition(pe_ctx* ctx, const int32_t* member_of_level, int n_levels, void* stream);

/* Copy a state in leaf layout (device) into the bound state (slot layout), and back. */
pe_status pe_set_state(pe_ctx* ctx, const double* u_leaf_dev, void* stream);
pe_status pe_get_state(pe_ctx* ctx, double* u_leaf_dev, void* stream);

/* Host copies of the slot -> leaf map and the member of every slot (each [n_elements]).
 * Either pointer may be NULL. */
pe_status pe_element_info(const pe_ctx* ctx, int32_t* leaf_of_slot, int32_t* member_of_slot);

/* The 1D Legendre-Gauss-Lobatto nodes on [-1, 1] and quadrature weights used by the DGSEM
 * (host arrays of degree+1 entries each; either may be NULL). */
pe_status pe_quadrature(const pe_ctx* ctx, double* nodes, double* weights);

/* The 2:1 mortar operators (Sec. 6.2; Kopriva's conservative mortars), host arrays
 * [2][N][N] each (either may be NULL), N = degree + 1: P[m][j][k] = l_k((x_j - 1)/2) (m = 0) or
 * l_k((x_j + 1)/2) (m = 1) interpolates the coarse face's nodal values to the nodes of half face
 * m; R[m] is the L2 projection (exact integrals) of nodal data on half face m back to the coarse
 * face, so that sum_m R[m] P[m] = I and sum_j w_j (R[m] g)_j = 1/2 sum_j w_j g_j (conservation).
 * In 3D the face operators are tensor products of these (factor 1/4 instead of 1/2). */
pe_status pe_mortar_operators(const pe_ctx* ctx, double* P, double* R);

/* Physical coordinates of every node in leaf layout, x_dev [leaf][dim][node] (device). */
pe_status pe_node_coords(pe_ctx* ctx, double* x_leaf_dev, void* stream);

/* du = F(u) on every element (both in slot layout, device; u may be the bound state).
 * The DGSEM right-hand side of Sec. 6.1 (flux-differencing volume integral, surface and
 * mortar fluxes, lifting; BR1 for Navier-Stokes). */
pe_status pe_rhs(pe_ctx* ctx, const double* u_dev, double* du_dev, void* stream);

/* Advance the bound state by n_steps partitioned P-ERK steps of size dt (eq.
 * PartitionedRKSystem with the tableaux of Sec. 3): stage i evaluates the right-hand side
 * only on the elements of the members that use stage i (a prefix of the slots); the
 * right-hand side of the other elements is never computed.  Asynchronous.  Unless graph replay
 * is off or profiling is on, the step's launches are captured once into a HIP graph and
 * replayed on `stream`; when the graph has to be captured again, the call's first step goes
 * out as plain launches and the capture runs on the host while they execute.  Should a capture
 * fail, the context continues with plain launches (graph replay off). */
pe_status pe_step(pe_ctx* ctx, double dt, int n_steps, void* stream);

/* pe_step replays one captured step as a HIP graph (captured again after every partition,
 * binding, coefficient or dt change) when on != 0 (default), or enqueues every launch when 0.
 * Results are identical either way. */
pe_status pe_set_graph_replay(pe_ctx* ctx, int on);

/* Element right-hand-side evaluations performed so far (device counter, read synchronously
 * on `stream`) in total and per member (out_per_member may be NULL, else [R]).  Multiplying by
 * n_vars * N^dim gives N_RHS^Actual of eq. (ActualRHSEvals).  reset != 0 zeroes them. */
pe_status pe_counters(pe_ctx* ctx, int64_t* out_total, int64_t* out_per_member, int reset,
                      void* stream);

/* ---------------------------------------------------------------- discrete adjoint (Euler)
 * Reverse mode of the partitioned step of Sec. 3.1 (Y_i = U_n + dt (a_{i,1} K_1 + a_{i,i-1}
 * K_{i-1}) with each element's member coefficients, K_i = I_i F(Y_i), U_{n+1} = U_n + dt
 * sum_i b_i K_i) and of the DGSEM right-hand side F of Sec. 6.1: derivatives of the computed
 * map, flux branches (HLL wave speeds, logarithmic-mean series) as the values take them. */

/* out = F'(u)^T w for the Euler right-hand side; u, w, out device arrays in slot layout
 * (n_state doubles, see pe_query_sizes; out must not alias u or w).  Asynchronous on stream.
 * PE_EUNSUPPORTED for Navier-Stokes. */
pe_status pe_rhs_vjp(pe_ctx* ctx, const double* u, const double* w, double* out, void* stream);

/* Device bytes of the adjoint workspace (S + 2 state arrays: the stage values of a
 * recomputed step and the stage cotangents), valid for the current coefficients and
 * capacity; pe_adjoint_bind hands over caller-owned memory (256-byte aligned). */
pe_status pe_adjoint_query(const pe_ctx* ctx, int64_t* bytes);
pe_status pe_adjoint_bind(pe_ctx* ctx, void* workspace);

/* lam_prev = Phi'(u_n)^T lam_next for one partitioned step Phi of size dt from u_n (slot
 * layout device arrays; lam_prev must not alias the inputs).  Recomputes the step from u_n,
 * keeping the stage values in the adjoint workspace, then sweeps the stages backwards
 * launching the adjoint kernel only on each stage's active elements and their face
 * neighbours.  The bound state is not touched; the stage workspace of pe_step is reused.
 * Asynchronous on stream. */
pe_status pe_step_adjoint(pe_ctx* ctx, double dt, const double* u_n, const double* lam_next, double* lam_prev,
                          void* stream);

/* A step's record for a later reverse sweep: K_1 and the stage values Y_2..Y_S (Sec. 3.1),
 * S state arrays, pe_adjoint_record_size doubles (device memory owned by the caller). */
pe_status pe_adjoint_record_size(const pe_ctx* ctx, int64_t* doubles);

/* One partitioned step of size dt from u_n into u_next, keeping its record (slot layout
 * device arrays; none may overlap another).  The same stage launches as pe_step; the bound
 * state is not touched, the stage workspace of pe_step is reused (it holds nothing between
 * steps).  Needs the adjoint workspace (pe_adjoint_bind); Euler only.  Asynchronous on
 * stream. */
pe_status pe_step_record(pe_ctx* ctx, double dt, const double* u_n, double* u_next, double* record, void* stream);

/* pe_step_adjoint from a record made by pe_step_record with the same u_n and dt, instead of
 * recomputing the step: bitwise the same lam_prev.  For checkpointed trajectories whose
 * segments are recomputed anyway (each step is then computed once, not twice). */
pe_status pe_step_adjoint_recorded(pe_ctx* ctx, double dt, const double* u_n, const double* record,
                                   const double* lam_next, double* lam_prev, void* stream);

/* Step-size bound of eq. (CFL_DG) and eq. (TimestepConstraint) from the bound state:
 * beta_l = 1 / max over the elements of level l, their nodes and the directions d of
 * (k+1)(|v_d| + c) / h_d  (k the polynomial degree, c the speed of sound; convective part only,
 * the bound the paper uses for its convection-dominated cases), and dt_out = cfl * min_l beta_l.
 * beta_of_level may be NULL, else [16] host doubles (0 for levels without elements).
 * Synchronises `stream`.  PE_ENONFINITE if the state gives a non-finite speed, PE_EINVAL if
 * cfl <= 0. */
pe_status pe_max_dt(pe_ctx* ctx, double cfl, double* dt_out, double* beta_of_level, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops): the
 * bound of pe_max_dt computed entirely on the device, with its scratch (one double per element
 * plus the 16 per-level maxima) in the library's static per-device array instead of the bound
 * workspace, and no allocation, copy to the host or synchronisation.  dt_dev [1] and beta_dev
 * [16] (may be NULL) are caller-owned device arrays written asynchronously on `stream`: the same
 * values pe_max_dt returns, except that a non-finite or all-zero wave speed gives dt = NaN
 * instead of an error.  At most 1048576 elements (PE_EINVAL beyond); PE_ESTATE without a
 * partition and a state, PE_EINVAL for a null dt_dev or cfl <= 0.  Every call on a device
 * shares that device's scratch: calls that overlap in time on one device (other streams, other
 * threads) race and must be ordered by the caller. */
pe_status pe_max_dt_noalloc(pe_ctx* ctx, double cfl, double* dt_dev, double* beta_dev, void* stream);

/* Which refinement indicator pe_amr_indicator and pe_amr_cycle compute (the paper's indicators
 * are cited in Sec. 7):
 *   PE_INDICATOR_DENSITY_GRADIENT (default; the adaptive Kelvin-Helmholtz workload):
 *     eta_e = h_e max_nodes |grad rho| / max_nodes rho; variable and f_wave are ignored;
 *   PE_INDICATOR_LOHNER (Loehner's indicator, the shear-layer workload of Sec. 7.1.1 on v_x):
 *     the largest |q_{i+1} - 2 q_i + q_{i-1}| / (|q_{i+1} - q_i| + |q_i - q_{i-1}|
 *     + f_wave (|q_{i+1}| + 2 |q_i| + |q_{i-1}|)) over the interior nodes of every coordinate line
 *     of the element's LGL nodes (three consecutive nodal values as they are; 0 where the
 *     denominator vanishes), q the primitive variable `variable` (0 rho, 1..dim the velocity
 *     components, dim+1 the pressure).
 *   PE_INDICATOR_HENNEMANN_GASSNER (the shock-capturing indicator, which the paper's
 *     Kelvin-Helmholtz run of Sec. 7.2.1 also uses for refinement; 2D, variable 0 = density only):
 *     1 / (1 + exp(-(s/T) (E - T))), E the energy share of the density's top modes as in
 *     pe_set_shock_capturing, without the cut-off and the cap; f_wave is ignored.
 * PE_EINVAL for another kind, a variable outside [0, dim+1] (HENNEMANN_GASSNER: not 0) or
 * f_wave < 0; PE_EUNSUPPORTED for HENNEMANN_GASSNER in 3D. */
typedef enum {
  PE_INDICATOR_DENSITY_GRADIENT = 0,
  PE_INDICATOR_LOHNER = 1,
  PE_INDICATOR_HENNEMANN_GASSNER = 2
} pe_indicator;
pe_status pe_set_amr_indicator(pe_ctx* ctx, int kind, int variable, double f_wave);

/* Subcell shock capturing (Hennemann, Rueda-Ramirez, Hindenlang and Gassner; the paper runs its
 * inviscid Kelvin-Helmholtz case with it, Sec. 4.1 and 7.2.1), 2D Euler.  At every right-hand-side
 * evaluation each element gets a blending factor alpha from its own stage value: with m_ab the
 * density's coefficients in the L2-orthonormal Legendre basis (V^-1 of the Vandermonde matrix of
 * sqrt(k + 1/2) P_k at the LGL nodes, applied per direction), all = sum m_ab^2, clip_k = the sum
 * over max(a, b) <= p - k, E = max((all - clip_1)/all, (clip_1 - clip_2)/clip_1),
 * T = 0.5 10^(-1.8 (p+1)^(1/4)), s = ln((1 - 1e-4)/1e-4): alpha = 1/(1 + exp(-(s/T)(E - T))),
 * 0 below alpha_min, at most alpha_max.  The volume term becomes (1 - alpha) times the
 * flux-differencing one plus alpha times first-order finite volumes on the LGL subcells:
 * (F_{i+1/2} - F_{i-1/2}) / w_i along each coordinate line, F the HLL flux of the two
 * neighbouring nodes, no subcell flux at the element's faces (the surface term is unchanged).
 * on = 0 switches it off (parameters ignored).  The next pe_step captures its graph again.
 * PE_EUNSUPPORTED for 3D, Navier-Stokes or an alternative stage pattern; PE_EINVAL unless
 * 0 <= alpha_min <= alpha_max <= 1.  While on, the tangent, the adjoint and the batched form
 * refuse the context, and pe_set_perk_coefficients a coupling table (PE_EUNSUPPORTED). */
pe_status pe_set_shock_capturing(pe_ctx* ctx, int on, double alpha_max, double alpha_min);

/* Refinement indicator per leaf (the one pe_set_amr_indicator selected; the density gradient by
 * default).  Written to eta_leaf_host [n_elements] in leaf order; synchronises `stream`.  (The
 * mesh change and re-flagging it triggers is Sec. 6.2.) */
pe_status pe_amr_indicator(pe_ctx* ctx, double* eta_leaf_host, void* stream);

/* Adapt the forest (Sec. 6.2: the mesh change after which the partition is rebuilt).
 * flags_host[n_elements] in leaf order: +1 refine, -1 coarsen, 0 keep; levels stay in
 * [level_min, level_max].  Rules: flagged leaves below level_max are refined once; coarser
 * face neighbours are refined until face neighbours differ by at most one level; a complete
 * family of 2^dim sibling leaves is coarsened only if all are flagged -1, none was refined,
 * their level exceeds level_min and no face neighbour outside the family ends finer than the
 * family's level.  The state is projected on the device (children: interpolation of the
 * parent polynomial; parents: LGL-quadrature L2 projection of the children, conservative).
 * The new leaf list is in Morton order (pe_get_leaves).  pe_partition must be called before
 * the next step.  PE_ENOMEM if the new mesh exceeds the reserved capacity (mesh unchanged). */
pe_status pe_adapt(pe_ctx* ctx, const int8_t* flags_host, int level_min, int level_max, void* stream);

/* One adaptation cycle in a single call (Sec. 6.2: indicator, mesh change, re-partition):
 * pe_amr_indicator; flags by threshold, +1 where eta > refine_above, then -1 where
 * eta < coarsen_below, 0 elsewhere (a NaN indicator keeps its leaf); pe_adapt with
 * [level_min, level_max]; pe_partition with member_of_level[n_levels] (NULL: the context's
 * level rule at the finest level of the adapted mesh).  The same flags,
 * forest and state as those calls made one by one.  flags_host (may be NULL) receives the
 * flags [n_elements before the call]; n_leaves (may be NULL) the number of leaves after it.
 * Synchronises `stream` once (the indicator download).  Errors as the three calls; on a
 * failure of pe_partition the forest is already adapted (call pe_partition again). */
pe_status pe_amr_cycle(pe_ctx* ctx, double refine_above, double coarsen_below, int level_min, int level_max,
                       const int32_t* member_of_level, int n_levels, int8_t* flags_host, int64_t* n_leaves,
                       void* stream);

/* Current leaf list (host) [n][4] (level, i, j, k); leaves may be NULL to query n. */
pe_status pe_get_leaves(const pe_ctx* ctx, int32_t* leaves, int64_t* n);

/* ---------------------------------------------------------------- spectrum estimation
 * Building blocks of the Arnoldi iteration on the Jacobian J = F'(u) of the right-hand side at
 * the real mesh (Sec. 4.1, steps 3-4: outer eigenvalues near scaled hull points of a reduced
 * spectrum).  Vectors are state arrays in slot layout (n = n_state_doubles of pe_query_sizes);
 * the iteration itself (basis, Hessenberg matrix, Ritz values) is driven by the caller.  The
 * product with J^T is pe_rhs_vjp (Euler; J^T has the eigenvalues of J). */

/* Directional derivative F'(u) v by central differences,
 * (F(u + h v) - F(u - h v)) / (2 h) with h = eps |u|_2 / |v|_2 (truncation O(h^2), any equations).
 * u, v, out: device state arrays (out must not alias u or v); uses the stage buffers of the
 * bound workspace as temporaries (they hold nothing between steps).  Synchronises `stream`
 * once.  PE_ESTATE before pe_partition; PE_EINVAL for eps <= 0, a zero v or null pointers. */
pe_status pe_rhs_jvp_fd(pe_ctx* ctx, const double* u, const double* v, double eps, double* out, void* stream);

/* Exact directional derivative t = F'(u) v of the Euler right-hand side (forward mode: every
 * quantity of the operator of Sec. 6.1 carried with its derivative; flux branches -- HLL wave
 * speeds and cases, the logarithmic-mean series -- as the values take them, a tie of the wave
 * speeds' min / max taking the first argument).  Optionally also f = F(u) (f may be NULL).
 * u, v, t, f: device state arrays in slot layout; t and f must not alias u or v.  Writes the
 * element slots only.  Asynchronous on `stream`.  PE_ESTATE before pe_partition,
 * PE_EUNSUPPORTED for Navier-Stokes, PE_EINVAL for null u, v or t. */
pe_status pe_rhs_jvp(pe_ctx* ctx, const double* u, const double* v, double* t, double* f, void* stream);

/* Device doubles of scratch pe_orthogonalize needs for k basis vectors. */
pe_status pe_orthogonalize_scratch(int k, int64_t* doubles);

/* One orthogonalisation of the Arnoldi iteration: w (device, n doubles) is orthogonalised
 * against the k columns of V (device; column j at V + j ldv, assumed orthonormal) by two passes
 * of classical Gram-Schmidt.  h_host [k + 1] receives the projections summed over both passes
 * and, in h_host[k], the norm of what is left, by which w is then divided (unless it is 0).
 * scratch: device, pe_orthogonalize_scratch(k) doubles.  Synchronises `stream`.  PE_EINVAL for
 * k < 0, n <= 0, ldv < n or null pointers. */
pe_status pe_orthogonalize(pe_ctx* ctx, const double* V, int k, int64_t ldv, double* w, int64_t n, double* scratch,
                           double* h_host, void* stream);

/* Self-check of the arithmetic routines the kernels use instead of library calls: the node
 * logarithms of the logarithmic means of the entropy-conserving flux (Sec. 6.1 volume flux),
 * the sound-speed square roots of the HLL wave speeds and the reciprocals.  For device arrays
 * x [n] and out [3n]: out[0, n) = ln x, out[n, 2n) = sqrt x, out[2n, 3n) = 1/x, asynchronous on
 * `stream`.  Meant for positive normal arguments (the kernels' domain): the logarithm of x <= 0
 * is NaN, the rest follow the hardware estimates.  PE_EINVAL for n < 0 or a null array with
 * n > 0. */
pe_status pe_device_math(pe_ctx* ctx, const double* x, int64_t n, double* out, void* stream);

/* Time every stage-kernel launch (and, for Navier-Stokes, every BR1 gradient launch) of pe_step
 * with a pair of HIP events recorded on the launch stream (on != 0), or stop (0).  Switching
 * resets the statistics. */
pe_status pe_set_profiling(pe_ctx* ctx, int on);

/* Sum of the event-measured durations of the stage kernels launched since profiling was
 * switched on (milliseconds; waits for the recorded events), the number of launches, and the
 * number of element-stages (active elements summed over the launches). */
pe_status pe_profile_stats(pe_ctx* ctx, double* kernel_ms, int64_t* launches, int64_t* element_stages);

/* The same per kernel: kernel 0 is the stage kernel (as pe_profile_stats), kernel 1 the BR1
 * gradient kernel (elements = active elements plus their inactive face neighbours, summed over
 * the launches), 2 the re-partitions of pe_amr_cycle (Sec. 6.2: the re-assignment of members
 * after a mesh change), each timed on the host from an idle stream to the end of its kernels
 * while profiling is on (launches = re-partitions, elements = elements re-partitioned).
 * PE_EINVAL for any other number. */
pe_status pe_profile_kernel_stats(pe_ctx* ctx, int kernel, double* kernel_ms, int64_t* launches, int64_t* elements);

/* ---------------------------------------------------------------- batched independent runs
 * Many independent partitioned P-ERK runs (the step of Sec. 3 with the level partition of
 * Sec. 6, each run with its own mesh, polynomial degree, coefficient family, stage count S and
 * dt) advanced together: one kernel launch per stage tick moves every unfinished run by one of
 * its own stages (one launch per polynomial degree present in the batch).  A run with S stages
 * and n steps is busy for n S ticks; tick t applies its stage t mod S.  The work of a tick is
 * the concatenation of the active element prefixes of the runs, cut into tiles; results are
 * bitwise those of pe_step on each run alone.
 * Supported: 2D Euler runs of degree 2 or 3 whose members all evaluate at least 3 stages.
 * Device tables for the batch are allocated by the library; the runs keep owning their state
 * and workspace, and pe_get_state / pe_counters read each run as usual. */

/* Group existing runs (each bound, with a state and a partition; at most once each).  The runs
 * must outlive the batch.  On failure *out is NULL and pe_batch_last_error(NULL) says why. */
pe_status pe_batch_create(pe_batch** out, pe_ctx* const* runs, int n_runs);
void pe_batch_destroy(pe_batch* batch);
const char* pe_batch_last_error(const pe_batch* batch);

/* Per run k: step dt[k] and number of steps n_steps[k] (host arrays [n_runs]).  Freezes the
 * runs' current partitions and buffers into device descriptors; call again after any change
 * to a run (adaptation, re-partition, new coefficients, re-binding).  Synchronous. */
pe_status pe_batch_set_steps(pe_batch* batch, const double* dt, const int64_t* n_steps);

/* Tile shape: elems_per_tile_p3 in {1, 2, 4} elements of degree 3 per tile (twice as many of
 * degree 2; a block of 64 * elems_per_tile_p3 lanes), grid_blocks blocks per tick (each block
 * takes every grid_blocks-th tile), or 0 for one block per tile. */
pe_status pe_batch_set_tiling(pe_batch* batch, int elems_per_tile_p3, int grid_blocks);

/* Number of ticks until every run has finished, and the element-stages they contain. */
pe_status pe_batch_info(const pe_batch* batch, int64_t* n_ticks, int64_t* element_stages);

/* Launch ticks [tick_begin, tick_end) on `stream` (asynchronous). */
pe_status pe_batch_run(pe_batch* batch, int64_t tick_begin, int64_t tick_end, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PERK_H */
