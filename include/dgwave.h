/*
 * dgwave.h -- C ABI of the MI355X (gfx950) nodal discontinuous Galerkin wave
 * step library.
 *
 * The library advances the semi-discrete nodal DG systems of Sec. 2 of
 * Modave, St-Cyr & Warburton, "GPU performance analysis of a nodal
 * discontinuous Galerkin method for acoustic and elastic models"
 * (arXiv:1602.07997):
 *   - acoustic pressure-velocity system with the upwind penalty of Sec. 2.1,
 *     right-hand side in the form of eqs. (5)-(6);
 *   - isotropic elastic velocity-stress system with the exact-Riemann upwind
 *     flux of Sec. 2.1 and the elastic right-hand side of Sec. 3.2 (the mu
 *     term read as 2 mu sym(grad v), as the PDE of Sec. 2.1 states);
 *   - anisotropic elastic velocity-stress system (a general symmetric
 *     positive definite Voigt stiffness per element; Sec. 5 names
 *     anisotropic media as future work), see DG_ANISOTROPIC below;
 *   - third-order Adams-Bashforth time stepping, eq. (4), started with one
 *     forward-Euler and one two-step Adams-Bashforth step.
 * The per-step work (volume term, face traces and upwind flux, merged LIFT,
 * AB3 update) runs in hand-written HIP kernels on one GPU.
 *
 * Conventions
 *   physics   DG_ACOUSTIC (fields p, v1, v2, v3), DG_ELASTIC or
 *             DG_ANISOTROPIC (fields v1, v2, v3, s11, s22, s33, s23, s13,
 *             s12).
 *   order     polynomial degree N, 1 <= N <= 8; Np = (N+1)(N+2)(N+3)/6 nodes
 *             per element, Nfp = (N+1)(N+2)/2 nodes per face.
 *   nodes     warp-and-blend nodes on the reference tetrahedron
 *             v1=(-1,-1,-1), v2=(1,-1,-1), v3=(-1,1,-1), v4=(-1,-1,1); node n
 *             is the lattice point with integer barycentrics (l1,l2,l3,l4),
 *             sum N, enumerated with l4 outermost, then l3, then l2.
 *   faces     f0=(v1,v2,v3), f1=(v1,v2,v4), f2=(v2,v3,v4), f3=(v1,v3,v4);
 *             face node j <-> (a,b) = barycentrics of the 2nd and 3rd face
 *             vertex, b outermost.
 *   fields    element-major float32 [K][Nfields][Np] (element k's block is
 *             contiguous; field c of element k starts at (k*Nfields + c)*Np).
 *   meshes    elem_xyz float64 [K][4][3] vertex coordinates, positively
 *             oriented; elem_topo int64 [K][4] topological vertex ids.  Two
 *             faces are neighbours iff they carry the same three ids; faces
 *             without a partner are reflecting walls (mirror ghost state:
 *             rigid wall for acoustics, traction-free for elasticity).
 *             Periodic boxes identify vertices through elem_topo while
 *             elem_xyz keeps unwrapped coordinates.  dg_set_boundary turns
 *             chosen unpaired faces into absorbing ones.
 *
 * Device memory: the library allocates none.  A solver, a batch and a misfit
 * each live in one caller-owned device buffer, the workspace, whose size the
 * matching *_workspace_bytes query gives (host-side, no GPU work); the buffer
 * must start on a 256-byte boundary (torch and hipMalloc allocations do),
 * must outlive the handle, and is used only by that handle.  The autotuner
 * takes a caller scratch array for its timed steps.  This follows the
 * paper's model of allocating everything once at start (Sec. 3.1).
 *
 * Pointers named "device" must point to GPU memory of the device current when
 * the solver was created; they are used stream-ordered on the solver's
 * stream, and the library keeps no reference to them after the call's work
 * has executed.  Pointers named "host" are read or written before the call
 * returns.  No call throws; every call returns a dg_status and on failure
 * dg_last_error() describes the cause (thread-local, valid until the next
 * failing call on the same thread).
 */
#ifndef DGWAVE_H
#define DGWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int dg_status;
#define DG_OK 0
#define DG_E_ARG (-1)         /* bad scalar argument or null pointer          */
#define DG_E_SHAPE (-2)       /* sizes inconsistent with the solver           */
#define DG_E_MESH (-3)        /* invalid mesh (orientation, connectivity)     */
#define DG_E_STATE (-4)       /* call out of order (e.g. step before fields)  */
#define DG_E_HIP (-5)         /* HIP runtime error                            */
#define DG_E_UNSUPPORTED (-6) /* degree or physics not built                  */
#define DG_E_UNSTABLE (-7)    /* non-finite or growing energy detected        */

#define DG_ACOUSTIC 0
#define DG_ELASTIC 1
/* Anisotropic elasticity (Sec. 5 lists it as future work; the reading is
 * this library's): rho dv/dt = div s, ds/dt = C e(v), s and the engineering
 * strain e in Voigt order (11, 22, 33, 23, 13, 12), C symmetric positive
 * definite.  Volume terms as the elastic right-hand side of Sec. 3.2 with C
 * in place of lambda, mu.  Upwind flux: the Riemann solution of media whose
 * waves all travel with one impedance per side, Z = sqrt(rho max_a C_aa)
 * (the P impedance for an isotropic C), applied to every traction and
 * velocity component; it dissipates (Z- Z+/(Z- + Z+)) |[v]|^2 + |[t]|^2 /
 * (Z- + Z+) per unit face area.  Walls and absorbing faces as DG_ELASTIC.
 * DG_VARIANT_VALU and DG_VARIANT_MFMA (FP32 matrix cores) are built for it;
 * the split 16-bit and element variants, and misfits, are not.             */
#define DG_ANISOTROPIC 2

typedef struct dg_solver dg_solver;

/* Version of this ABI (bumped on any incompatible change). */
int dg_abi_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* dg_last_error(void);

/* Number of fields for a physics (4 acoustic, 9 elastic and anisotropic),
 * or -1. */
int dg_num_fields(int physics);

/* ------------------------------------------------------------------------ */
/* Host-only set-up queries (no GPU needed).                                */
/* ------------------------------------------------------------------------ */

/* Np and Nfp for degree `order` (1..8).  Np/Nfp are host int*. */
dg_status dg_ref_sizes(int order, int* Np, int* Nfp);

/* Reference element of degree `order` (Sec. 2.2: nodal expansion eq. (1),
 * differentiation matrices D_j and merged lift matrix L of eqs. (3), (5)-(6)),
 * all host arrays owned by the caller, row-major, any of them may be NULL:
 *   nodes [Np][3]          (r,s,t) of the warp-and-blend nodes
 *   D     [3][Np][Np]      D[j][n][m] = d ell_m / d r_j at node n
 *   mass  [Np][Np]         reference mass matrix (volume 4/3)
 *   lift  [Np][4*Nfp]      merged LIFT = M^{-1}[E_0..E_3], face blocks in
 *                          face order, face mass in the parameter triangle
 *                          (-1,-1),(1,-1),(-1,1) through the face's vertices
 *   fmask [4][Nfp]         volume node of face node j of face f            */
dg_status dg_reference_operators(int order, double* nodes, double* D, double* mass,
                                 double* lift, int32_t* fmask);

/* Face-node permutation for the six relative orientations of two faces that
 * share three vertices (the per-face-node neighbour map of Sec. 3.2, stored
 * per face instead of per node).  perm is host int32 [6][Nfp]: own face node j
 * meets neighbour face node perm[o][j], where o indexes the permutation pi of
 * the face's vertices (own vertex p is neighbour vertex pi(p)) in the order
 * (0,1,2),(0,2,1),(1,0,2),(1,2,0),(2,0,1),(2,1,0).                         */
dg_status dg_face_permutations(int order, int32_t* perm);

/* Face connectivity of a mesh from its topological ids (host arrays):
 *   e2e [K][4] neighbour element or -1 (wall); e2f [K][4] neighbour face or
 *   -1; orient [K][4] orientation index (see dg_face_permutations) or -1.
 * Fails with DG_E_MESH if a face is shared by more than two elements or an
 * element repeats a vertex id.                                              */
dg_status dg_mesh_connectivity(int64_t K, const int64_t* elem_topo, int64_t* e2e, int32_t* e2f,
                               int32_t* orient);

/* ------------------------------------------------------------------------ */
/* Solver (needs a GPU).                                                    */
/* ------------------------------------------------------------------------ */

/* Bytes of device workspace a solver of this physics, degree and element
 * count needs (*bytes, host): fields, the AB3 ring of eq. (4), trace
 * buffers, geometry and coefficient arrays and the operator tables of
 * eqs. (5)-(6) in every kernel layout.  Host-only; no GPU needed.  Errors:
 * DG_E_ARG (unknown physics, K outside [1, 2^26), null output),
 * DG_E_UNSUPPORTED (order outside [1, 8]).                                  */
dg_status dg_workspace_bytes(int physics, int order, int64_t K, size_t* bytes);

/* Create a solver for `K` elements of degree `order`.  elem_xyz (host
 * float64 [K][4][3]) and elem_topo (host int64 [K][4]) are copied; the
 * geometry (per-element inverse Jacobian G[i][j] = d r_j / d x_i, the volume
 * factor of eq. (3); face normals and Fscale = sJ/J, the surface factor) and
 * connectivity are built on the host in float64 and uploaded, together with
 * the reference operators (uploaded once, Sec. 3.1), into `workspace`
 * (device, workspace_bytes >= dg_workspace_bytes, 256-byte aligned, owned by
 * the caller, outliving the solver).  `stream` is a hipStream_t (NULL =
 * default stream) used by every later call; the call synchronises it.  K must
 * lie in [1, 2^26) (the per-face connectivity word packs the neighbour index
 * in 26 bits).  Two launch options are read from the environment here,
 * neither of which changes any result: DGWAVE_XCD_REMAP=1 gives each XCD a
 * contiguous range of tiles (default: launch order), DGWAVE_TAIL_SPLIT=0
 * keeps the tiles of a short last round of MFMA workgroups whole (default:
 * shared by two or three workgroups where a tile has more (node block,
 * element block) pairs than wavefronts).  Errors: DG_E_ARG (K out of range,
 * null or misaligned arrays), DG_E_SHAPE (workspace too small),
 * DG_E_UNSUPPORTED, DG_E_MESH (J <= 0, inconsistent face pairing), DG_E_HIP. */
dg_status dg_create(int physics, int order, int64_t K, const double* elem_xyz,
                    const int64_t* elem_topo, void* workspace, size_t workspace_bytes, void* stream,
                    dg_solver** out);

/* Release the solver (synchronises its stream); its workspace is the
 * caller's to free afterwards. */
void dg_destroy(dg_solver* s);

/* Replace the stream used by later calls (hipStream_t, NULL = default). */
dg_status dg_set_stream(dg_solver* s, void* stream);

/* Kernel variant of the step (default DG_VARIANT_VALU).  All compute the
 * right-hand side of eqs. (5)-(6) / the elastic system and the update of
 * eq. (4); they differ in how the D_j and LIFT products run:
 *   DG_VARIANT_VALU       node per thread, vector ALU;
 *   DG_VARIANT_MFMA       element tiles on FP32 matrix cores;
 *   DG_VARIANT_MFMA_BF16  BF16 matrix cores with FP32 accumulation, both
 *                         operands split x = x_hi + x_lo and the products
 *                         D_hi x_hi + D_hi x_lo + D_lo x_hi;
 *   DG_VARIANT_MFMA_F16   the same with FP16 halves, which need field and
 *                         face-penalty values well inside FP16's range: a
 *                         value beyond 65504 overflows (the results turn
 *                         non-finite and dg_energy reports DG_E_UNSTABLE),
 *                         and below about 1e-3 the lo half is subnormal and
 *                         the products lose accuracy (O(1) amplitudes give
 *                         the 1e-5 relative accuracy of the other variants);
 *   DG_VARIANT_ELEM       one element per thread, all in registers
 *                         (acoustic N = 1, 2; elastic N = 1);
 *   DG_VARIANT_MFMA_WIDE  FP32 matrix cores with the other acoustic tile
 *                         shape: twice the elements and wavefronts per
 *                         workgroup from N = 4, half the elements below
 *                         (acoustic only), a tile-shape candidate for
 *                         dg_autotune (the paper tunes its elements per
 *                         block per degree, Sec. 3.2 and Table 5).
 * The VALU and MFMA variants are built for the acoustic and elastic physics
 * and N = 1..8; the anisotropic physics has DG_VARIANT_VALU and
 * DG_VARIANT_MFMA.
 * Fields, r and the update stay FP32 in every variant.  Returns
 * DG_E_UNSUPPORTED for a combination that is not built.                    */
#define DG_VARIANT_VALU 0
#define DG_VARIANT_MFMA 1
#define DG_VARIANT_MFMA_BF16 2
#define DG_VARIANT_MFMA_F16 3
#define DG_VARIANT_ELEM 4
#define DG_VARIANT_MFMA_WIDE 5
dg_status dg_set_variant(dg_solver* s, int variant);
dg_status dg_get_variant(dg_solver* s, int* variant);

/* Wait for all work queued by the solver. */
dg_status dg_synchronize(dg_solver* s);

/* Physical coordinates of every node, host float64 [K][Np][3]. */
dg_status dg_node_coordinates(dg_solver* s, double* xyz);

/* Material coefficients per element, device float32: acoustic [K][2]
 * (rho, c); elastic [K][3] (rho, lambda, mu), all > 0 (mu > 0 is required by
 * the elastic flux); anisotropic [K][22] (rho > 0, then the 21 entries C_ab,
 * a <= b, of the upper triangle of the Voigt stiffness row by row: C_00 ..
 * C_05, C_11 .. C_15, ..., C_55; C positive definite).  Validated on the
 * device (synchronises); derived per-face impedances of the neighbours are
 * computed on the device.  Must precede dg_step/dg_rhs.  Errors: DG_E_ARG
 * (null, a value that is not positive and finite, or an anisotropic
 * stiffness that is not finite and positive definite in double precision:
 * the solver then has no coefficients until the next successful call),
 * DG_E_HIP.                                                                 */
dg_status dg_set_coefficients(dg_solver* s, const float* coef);

/* Kind of each unpaired face, host int32 [K][4]: DG_BC_REFLECT (the default
 * of dg_create: mirror ghost state, rigid wall for acoustics, traction-free
 * for elasticity) or DG_BC_ABSORB.  Sec. 5 lists artificial boundary
 * conditions as future work; the reading here: an absorbing face sees a
 * zero exterior state with the element's own coefficients, so that the
 * upwind flux of Sec. 2.1 lets no characteristic enter (acoustic alpha
 * becomes -(p - Z v.n)/2 of the element's own trace).  Entries of faces that
 * have a neighbour must be DG_BC_REFLECT.  May be called at any time (the
 * next step uses it); the misfit gradient supports both kinds.  Synchronises
 * the solver's stream.  Errors: DG_E_ARG (null, an unknown kind, an
 * absorbing face that has a neighbour), DG_E_HIP.                           */
#define DG_BC_REFLECT 0
#define DG_BC_ABSORB 1
dg_status dg_set_boundary(dg_solver* s, const int32_t* kind);

/* Set the fields (device float32 [K][Nfields][Np]); resets the step counter
 * to 0 so that the next steps use the Euler / two-step start-up.            */
dg_status dg_set_fields(dg_solver* s, const float* q);

/* Copy the current fields to device float32 [K][Nfields][Np]. */
dg_status dg_get_fields(dg_solver* s, float* q);

/* Full AB3 state for checkpoint / resume: q^m, r^{m-1}, r^{m-2} (device
 * float32, each [K][Nfields][Np]; r1/r2 ignored when step_index < 1 / < 2)
 * and the step index m.  DG_E_UNSUPPORTED on a two-rate solver.             */
dg_status dg_set_state(dg_solver* s, const float* q, const float* r1, const float* r2,
                       int64_t step_index);
dg_status dg_get_state(dg_solver* s, float* q, float* r1, float* r2, int64_t* step_index);

/* Current step index m (host int64*). */
dg_status dg_step_index(dg_solver* s, int64_t* m);

/* Advance `nsteps` steps of size dt (eq. (4)); one fused kernel per step,
 * asynchronous on the solver's stream.  Errors: DG_E_ARG, DG_E_STATE (no
 * coefficients or fields, or a fast class set: see dg_step_multirate).      */
dg_status dg_step(dg_solver* s, int nsteps, double dt);

/* Two-rate (local) time stepping, which Sec. 1 names as an advantage of DG
 * and Sec. 5 calls essential for large meshes without giving a scheme; the
 * reading here: elements [0, k_fast) form a fast class that takes two steps
 * of dt/2 per step dt of the slow class [k_fast, K) (the caller orders the
 * elements so, e.g. by local CFL step).  Each class runs eq. (4) with its
 * own right-hand-side history and Euler / two-step start-up.  Per macro
 * step: (1) fast half step from t_n; (2) slow full step from t_n; (3) the
 * traces at t_n + dt/2 of the slow elements next to fast ones, from the
 * integral of their Adams-Bashforth history polynomial over the half step
 * (17/24, -7/24, 1/12 in AB3, the half-step analogue of eq. (4)'s
 * weights); (4) fast half step from t_n + dt/2.  dg_set_rate_classes sets
 * the split (k_fast in [0, K]; 0 = single rate) and restarts the start-up;
 * it synchronises.  A solver with k_fast > 0 steps only with
 * dg_step_multirate (dg_step, dg_set_state, dg_get_state and batches refuse
 * it: its history is per class); dg_step_multirate with k_fast = 0 is
 * dg_step.  The step index counts macro steps.  Errors: DG_E_ARG,
 * DG_E_STATE (no coefficients or fields), DG_E_HIP.                         */
dg_status dg_set_rate_classes(dg_solver* s, int64_t k_fast);
dg_status dg_step_multirate(dg_solver* s, int nsteps, double dt);

/* One evaluation of the right-hand side r(q) of eqs. (2)-(3): q and r are
 * device float32 [K][Nfields][Np]; does not touch the solver's state.       */
dg_status dg_rhs(dg_solver* s, const float* q, float* r);

/* Discrete energy of the current fields, accumulated in float64 on the GPU:
 * acoustic 1/2 sum_k J_k [p^T M p/(rho c^2) + rho sum_i v_i^T M v_i];
 * elastic 1/2 sum_k J_k [rho sum_i v_i^T M v_i + (s:s - lambda/(3 lambda +
 * 2 mu) tr(s)^2)/(2 mu)] with the mass matrix (off-diagonal stresses twice).
 * Synchronises; *e is host float64.  Stability check: the upwind flux of
 * Sec. 2.1 only dissipates, so returns DG_E_UNSTABLE (with *e set) if the
 * energy is not finite, or if it exceeds (1 + tol) times the previous
 * dg_energy result of the same trajectory, both evaluations in the AB3
 * regime (step index >= 2; dg_set_fields / dg_set_state start a new
 * trajectory).  tol defaults to 1e-4, see dg_set_energy_tolerance.          */
dg_status dg_energy(dg_solver* s, double* e);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the energy
 * of dg_energy, computed by the same kernels, written to the device float64
 * *e_dev on the solver's stream without synchronising, without a host copy
 * and without the growth check.  The per-workgroup partial sums go to a
 * static device array of the library (16384 float64, 128 KiB, one per
 * device, held until the process ends) instead of the solver's buffers; the
 * call allocates nothing.  Meshes that need more partial sums than that
 * (elements per energy workgroup: 64 at N = 1 down to 3 at elastic N = 6,
 * e.g. acoustic N = 5 beyond 65536 elements) get DG_E_SHAPE.  Every call on
 * one device shares that array: calls that overlap on one GPU (from
 * different streams or threads) race and may return wrong sums; calls on one
 * stream are ordered and safe.  Errors: DG_E_ARG (null e_dev), DG_E_SHAPE,
 * DG_E_STATE (no coefficients or fields), DG_E_HIP.                         */
dg_status dg_energy_noalloc(dg_solver* s, double* e_dev);

/* Growth tolerance of dg_energy's stability check (>= 0); a negative value
 * disables the growth check (non-finite energies are still flagged).
 * Errors: DG_E_ARG (NaN).                                                    */
dg_status dg_set_energy_tolerance(dg_solver* s, double tol);

/* Diagnostics: copy one internal device buffer of the solver into caller
 * memory (host), for layout and data checks in tests.  `name` is one of
 * "geo" (float32 [K][9]), "cf" (float32 [K][CB]), "conn" (int32 [K][4]),
 * "fmask" (int32 [4][Nfp]), "perm" (int32 [6][Nfp]), "nodeface" (int32
 * [Np][3], the face slots f*Nfp+j of each node, -1 padded), "DT" (float32
 * [3][Np][Np], DT[j][m][n] = D_j[n][m]), "LT" (float32 [4Nfp][Np]),
 * "traces" (float32 [K][4][NT][Nfp], the traces of the current fields) or
 * "traces_rhs" (traces of the last dg_rhs input).  *bytes is the buffer
 * size on return; nothing is copied when dst is NULL or *bytes is too small
 * on entry (DG_E_SHAPE).  Synchronises the solver's stream.               */
dg_status dg_debug_buffer(dg_solver* s, const char* name, void* dst, size_t* bytes);

/* ------------------------------------------------------------------------ */
/* Kernel choice and batches of meshes.                                     */
/* ------------------------------------------------------------------------ */

/* Time the kernel variants built for the solver's physics and degree on the
 * solver's own mesh: `steps` steps of size dt each with the AB3 weights of
 * eq. (4), after one untimed step, timed with HIP events on the solver's
 * stream.  `candidates` is a bit mask of the variants to consider (bit v for
 * variant v; 0 = all of them).  Every timed step reads the current state
 * and writes its fields into `scratch` (device, scratch_bytes >= K*Nfields*Np
 * float32), its r into the ring slot of r^{m-3} and its traces into the
 * buffer the next step overwrites, so the state (fields, AB3 history,
 * traces, step index) does not change; the call synchronises.  The fastest
 * variant becomes the solver's variant.
 * us_per_step (host float64 [DG_NUM_VARIANTS], may be NULL) receives the
 * microseconds per step of each variant, -1 where not built or not a
 * candidate.  The choice of
 * kernel per degree and mesh follows the observation of Sec. 4 that the best
 * implementation strategy depends on the degree.  The autotuner compares
 * speed only: leave the split 16-bit variants out of `candidates` unless the
 * fields suit them (see dg_set_variant).  Errors: DG_E_STATE (no
 * coefficients or fields), DG_E_ARG, DG_E_HIP.                              */
#define DG_NUM_VARIANTS 6
dg_status dg_autotune(dg_solver* s, int steps, double dt, unsigned candidates, void* scratch,
                      size_t scratch_bytes, double* us_per_step);

typedef struct dg_batch dg_batch;

/* A batch steps `count` independent solvers together: one kernel launch per
 * (degree, variant) group and step, over a device work list of (member,
 * element tile) pairs, instead of one launch per mesh.  members is a host
 * array of distinct solvers of one physics created on the current device;
 * the batch keeps the pointers (not ownership): every member must outlive
 * the batch.  Each member keeps its own buffers, coefficients and variant
 * (the groups are rebuilt when a member's variant changes).  `stream` is the
 * hipStream_t the batched work is ordered on (NULL = default stream): with
 * more than one group, each step forks onto one library-owned stream per
 * group (default priority) and joins back, so that the groups' launches
 * overlap; the members are independent meshes.  The work
 * lists and argument tables live in `workspace` (device, workspace_bytes >=
 * dg_batch_workspace_bytes, 256-byte aligned, owned by the caller and
 * outliving the batch).  Errors: DG_E_ARG (null, repeated or mixed-physics
 * members, bad workspace), DG_E_SHAPE (workspace too small), DG_E_HIP.      */
dg_status dg_batch_create(dg_solver* const* members, int count, void* workspace, size_t workspace_bytes,
                          void* stream, dg_batch** out);

/* Workspace bytes of a batch of these members (*bytes, host): enough for
 * every choice of their kernel variants.  Errors: DG_E_ARG.                 */
dg_status dg_batch_workspace_bytes(dg_solver* const* members, int count, size_t* bytes);

/* Release the batch (synchronises its stream; members are untouched). */
void dg_batch_destroy(dg_batch* b);

/* Record six consecutive batched steps in a HIP graph and replay it for
 * whole runs of six steps (enable = 1), or launch kernel by kernel (0, the
 * default).  The graph holds kernel nodes only, one independent chain of six
 * per launch group; it needs a non-NULL stream (DG_E_STATE otherwise).      */
dg_status dg_batch_set_graph(dg_batch* b, int enable);

/* Advance every member by `nsteps` steps of eq. (4); dt is host float64
 * [count], member i's step size.  Members still in the start-up (step index
 * below 2) take that step with their own launch; once all are in the AB3
 * regime the steps are batched.  Members may start at different step
 * indices.  Asynchronous on the batch's stream.  Errors: DG_E_ARG, DG_E_STATE
 * (a member without coefficients or fields), DG_E_HIP.                      */
dg_status dg_batch_step(dg_batch* b, int nsteps, const double* dt);

/* Shape of the batch.  On return *ngroups is the number of launch groups;
 * order, variant (host int32) and tiles (host int64, workgroups of the
 * group's launch) receive one entry per group.  When any array is non-NULL,
 * *ngroups on entry is their capacity (DG_E_SHAPE if too small); call with
 * NULL arrays first to ask for the count.                                   */
dg_status dg_batch_groups(dg_batch* b, int* ngroups, int32_t* order, int32_t* variant, int64_t* tiles);

/* ------------------------------------------------------------------------ */
/* Misfit and its coefficient gradient (adjoint).                           */
/* ------------------------------------------------------------------------ */

/* Locate n points (host float64 [n][3]) in the solver's mesh: elem (host
 * int64 [n]) the first element whose barycentric coordinates are all >=
 * -1e-12, weights (host float64 [n][Np], may be NULL) the nodal Lagrange
 * weights of the point (u(x) = weights . u_nodes; the expansion of eq. (1)).
 * DG_E_ARG if a point lies outside the mesh.                                  */
dg_status dg_locate_points(dg_solver* s, int64_t n, const double* xyz, int64_t* elem, double* weights);

typedef struct dg_misfit dg_misfit;

/* A least-squares problem on the solver's mesh and coefficients:
 *   forward: q^0 = 0, steps of eq. (4) of size dt with the point source
 *     f(t_m) b added to r^m, b = (1/J_k) M^{-1} l(x_s) (the projection of a
 *     Dirac mass) in the source fields: acoustic p, elastic s11, s22, s33;
 *     wavelet (host float64 [nsteps+1]) holds f(t_m), t_m = m dt;
 *   receivers: u(t_m) = l(x_r) . q in the recorded fields (acoustic p;
 *     elastic v1, v2, v3), channel index = receiver * fields + field;
 *   misfit: J = 1/2 dt sum_{m=1..nsteps} sum_channels (u - d)^2.
 * src_xyz / rec_xyz are host float64 [n][3].  The forward states are kept
 * every checkpoint_every steps; the gradient recomputes the steps between
 * checkpoints.  Its device arrays, about (checkpoint_every + 3 nsteps /
 * checkpoint_every + 9) field arrays, live in `workspace` (device,
 * workspace_bytes >= dg_misfit_workspace_bytes of the same arguments,
 * 256-byte aligned, owned by the caller and outliving the misfit).  The
 * solver must outlive the misfit; the misfit uses its own state buffers (the
 * solver's fields are not touched).  Errors: DG_E_ARG (bad sizes, a point
 * outside the mesh, bad workspace), DG_E_SHAPE (workspace too small),
 * DG_E_UNSUPPORTED (an anisotropic solver), DG_E_HIP.                       */
dg_status dg_misfit_create(dg_solver* s, int64_t nsteps, double dt, int checkpoint_every, int nsrc,
                           const double* src_xyz, const double* wavelet, int nrec, const double* rec_xyz,
                           void* workspace, size_t workspace_bytes, dg_misfit** out);

/* Workspace bytes of dg_misfit_create with the same arguments (*bytes,
 * host; locates the points on the host, no GPU work).  Errors as
 * dg_misfit_create's argument checks.                                       */
dg_status dg_misfit_workspace_bytes(dg_solver* s, int64_t nsteps, double dt, int checkpoint_every, int nsrc,
                                    const double* src_xyz, const double* wavelet, int nrec,
                                    const double* rec_xyz, size_t* bytes);
void dg_misfit_destroy(dg_misfit* f);

/* Number of receiver channels, or -1 for a NULL misfit. */
int64_t dg_misfit_channels(dg_misfit* f);

/* Forward solve with the solver's current coefficients.  data (device
 * float32 [nsteps+1][channels], may be NULL) is copied; traces (device
 * float32 [nsteps+1][channels], may be NULL) receives the receiver values;
 * *J (host, may be NULL) the misfit against data (0 without data; the call
 * then synchronises).  Errors: DG_E_STATE (no coefficients),
 * DG_E_UNSUPPORTED (the solver's variant is DG_VARIANT_MFMA_F16, whose FP16
 * operands cannot hold the projected point source), DG_E_UNSTABLE (J not
 * finite), DG_E_HIP.                                                        */
dg_status dg_misfit_forward(dg_misfit* f, const float* data, float* traces, double* J);

/* Gradient of J with respect to the per-element coefficients (acoustic
 * (rho, c), elastic (rho, lambda, mu)), device float32 [K][ncoef], by the
 * discrete adjoint of the forward steps (exact up to rounding): the reverse
 * recursion runs on the forward step kernel through A^T = P W A P W^{-1}
 * (W the energy weight, P = -1 on velocities), checkpointed segments are
 * recomputed, and the coefficient derivatives of the energy weight and of
 * the upwind penalty are accumulated per element in float64.  Needs a
 * preceding dg_misfit_forward with data; DG_E_STATE if there was none or if
 * dg_set_coefficients was called on the solver after it.  Errors:
 * DG_E_STATE, DG_E_UNSUPPORTED (as dg_misfit_forward), DG_E_HIP.           */
dg_status dg_misfit_gradient(dg_misfit* f, float* grad);

#ifdef __cplusplus
}
#endif

#endif /* DGWAVE_H */
