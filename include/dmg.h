/*
 * dmg.h -- C ABI of the MI355X (gfx950) structured multigrid library for remapped elliptic
 * problems.
 *
 * Method: Nytko, MacLachlan, Moulton, Olson, Reisner, West, "Unstructured to structured:
 * geometric multigrid on complex geometries via domain remapping" (arXiv 2509.08109).
 * A physical domain is pulled back through a diffeomorphism onto the logical square
 * (-1,1)^2 (Sec. 2, eq. weak_computational); there -div(K grad u) becomes a 9-point Q1 stencil
 * whose coefficients come from the map's metric det(J) J^{-1} J^{-T} (Sec. 2.1, effective
 * tensor D_c).  The structured system is solved by black-box multigrid V-cycles (Sec. 2.2):
 * factor-two coarsening, operator-induced interpolation, Galerkin coarse operators P^T A P.
 * Vectors move between a P1 mesh and the grid with the L2 projection P = M_p^{-1} C and its
 * transpose (Sec. 2.3).
 *
 * Conventions (all entry points):
 *  - Every array pointer is a DEVICE pointer owned by the caller unless stated otherwise.
 *    Arrays are dense, row-major, i (the xi index) fastest:
 *      vertex arrays [ny][nx] (boundary ring included), cell arrays [ny-1][nx-1].
 *  - Stencils use symmetric 5-value storage (Sec. 4.1, closing remark on storage):
 *      S[0]=C (diagonal), S[1]=W (coupling to (i-1,j)), S[2]=S (to (i,j-1)),
 *      S[3]=SW (to (i-1,j-1)), S[4]=SE (to (i+1,j-1)); each plane [ny][nx].
 *    The E, N, NE, NW couplings of (i,j) are W(i+1,j), S(i,j+1), SW(i+1,j+1), SE(i-1,j+1).
 *    Values are the matrix entries themselves (off-diagonals <= 0 for M-matrices).
 *    Dirichlet rows and all couplings into the boundary ring are zero.
 *  - Boundary entries of right-hand sides are ignored; boundary entries of solutions are
 *    written as 0 (homogeneous Dirichlet; inhomogeneous data is lifted by the caller).
 *  - Work is enqueued on the given hipStream_t (NULL = default stream) and is asynchronous,
 *    except for functions that return host scalars (they synchronise that stream).
 *  - Every function returns dmg_status; on failure dmg_last_error() (thread-local) holds a
 *    message.  Argument validation happens on the host before anything is enqueued, so a
 *    rejected call has no device side effects.  No C++ exception crosses this boundary.
 *  - Grid dimensions: any odd size >= 3 in each direction for the solver (dmg_setup states how
 *    levels coarsen and which coarsest grids are accepted); assembly accepts any size >= 3.
 */
#ifndef DMG_H
#define DMG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dmg_status {
  DMG_OK = 0,
  DMG_ERR_INVALID_ARG = 1,    /* null pointer, negative size, bad option value          */
  DMG_ERR_DIMS = 2,           /* grid dims even or < 3, coarsest grid too large          */
  DMG_ERR_WORKSPACE = 3,      /* workspace missing, misaligned (256 B) or too small        */
  DMG_ERR_NOT_SPD = 4,        /* coarsest-level Cholesky met a non-positive pivot          */
  DMG_ERR_NONFINITE = 5,      /* NaN/Inf in a residual norm                               */
  DMG_ERR_NO_CONVERGENCE = 6, /* max_iters reached before the tolerance                   */
  DMG_ERR_HIP = 7,            /* a HIP runtime call failed                                */
  DMG_ERR_UNSUPPORTED = 8
} dmg_status;

enum { DMG_FP64 = 0, DMG_FP32_IR = 1 };

/* Mesh setup flags (dmg_transfer_create_mesh, dmg_twolevel_create). */
enum {
  DMG_MESH_HOST_SETUP = 1, /* assemble C and C^T on the host instead of the device */
  DMG_MESH_MATRIX_FREE = 2 /* store no C: recompute its action from the overlap sets each apply */
};

/* Solver options.  Fill with dmg_default_options() and change what is needed. */
typedef struct dmg_options {
  int32_t nu_pre;        /* pre-smoothing sweeps per level (default 1)                    */
  int32_t nu_post;       /* post-smoothing sweeps per level (default 1)                   */
  int32_t pre_order[4];  /* colour order of a pre-smoothing sweep (default 0,1,2,3);
                            colour(i,j) = (i mod 2) + 2 (j mod 2); must be a permutation   */
  int32_t post_order[4]; /* colour order of a post sweep (default 3,2,1,0: the reverse,
                            which keeps the V-cycle symmetric)                             */
  int32_t coarsest_n;    /* stop coarsening when min(nx,ny) <= coarsest_n (default 3);
                            the coarsest interior system is solved by dense Cholesky       */
  int32_t precision;     /* DMG_FP64 (default) or DMG_FP32_IR                              */
  int32_t inner_cycles;  /* FP32 V-cycles per refinement step for DMG_FP32_IR (default 1) */
  int32_t use_graph;     /* capture one cycle in a hipGraph and replay it (default 1)      */
  int32_t tile_rows;     /* launch-shape knob of the fused sweep kernels; 0 = built-in
                            table.  Numerically neutral.                                   */
  int32_t strip_kernel;  /* implementation of the large-level sweeps before autotuning:
                            0 = LDS strips, 1 = one-wavefront strips (default 1).  The two
                            sum the stencil terms in different orders: their iterates agree
                            to rounding (~1e-14 relative), not bitwise.                     */
  int32_t smoother;      /* 0 = 4-colour point Gauss-Seidel (default, fused kernels);
                            zebra line Gauss-Seidel for anisotropic operators: 1 = x-lines
                            (rows), 2 = y-lines (columns), 3 = alternating x then y.  Each
                            interior line of one parity, even lines first, is solved exactly
                            with the other lines held; the post sweep runs in reverse (the
                            V-cycle stays symmetric).  Line smoothing runs unfused level by
                            level: in float64, in the float32 inner cycles of DMG_FP32_IR
                            (float32 stencils, weights and Thomas factors), and in the batch
                            solve (each line step launched once per level size over all
                            instances); nu_pre / nu_post count whole line sweeps.         */
  int32_t coarse_gemv;   /* 1 (default): when the coarse kernel's top level is a coarse level
                            with at most 1024 interior unknowns (33 x 33), apply the cycle from
                            there down as its dense matrix (built at setup) with one
                            matrix-vector product over the whole GPU; 0: the one-workgroup
                            coarse kernel.  The same cycle: only the rounding differs.  The
                            batch solver always uses 0 (its instances' matrices together would
                            cost more bandwidth than they save).                           */
  int32_t reserved[4];
} dmg_options;

typedef struct dmg_hier dmg_hier;
typedef struct dmg_transfer dmg_transfer;
typedef struct dmg_batch dmg_batch;
typedef struct dmg_twolevel dmg_twolevel;

void dmg_default_options(dmg_options* opts);
const char* dmg_last_error(void);
const char* dmg_version(void);

/* ---- stencil assembly (Sec. 2, eq. weak_computational; Sec. 2.1 D_c) --------------------
 * jac : [16][ny-1][nx-1] float64.  Plane 4*q+e is entry e of J = dX/d(xi,eta) of the inverse
 *       map X = T^{-1} (e = 0: dx/dxi, 1: dx/deta, 2: dy/dxi, 3: dy/deta) at the 2x2 Gauss point
 *       q = qx + 2 qy of each cell, local offsets 1/2 -+ 1/(2 sqrt 3) of the cell width.
 *       det J must be > 0.
 * K   : [ny-1][nx-1] float64 scalar diffusion coefficient per cell (D = K I).
 * S   : [5][ny][nx] float64 output: A = sum_cells K_e int grad phi_a . M grad phi_b,
 *       M = det(J) J^{-1} J^{-T}, with the 2x2 Gauss rule; Dirichlet rows/couplings zero.
 * nx, ny >= 3 (any size).  Errors: DMG_ERR_INVALID_ARG, DMG_ERR_DIMS, DMG_ERR_HIP. */
dmg_status dmg_assemble_stencil(const double* jac, const double* K, int32_t nx, int32_t ny,
                                double* S, hipStream_t stream);

/* ---- hierarchy setup (Sec. 2.2; coarsening by two, operator-induced interpolation,
 * Galerkin P^T A P, dense Cholesky of the coarsest interior system) --------------------------
 * The hierarchy lives entirely in a caller-provided device workspace (>= *bytes, 256-byte
 * aligned) which must outlive the handle; the library does not allocate device memory for it.
 * The fine stencil S is copied into the workspace (the caller may free it after setup).
 * Setup synchronises `stream` once to read the coarsest pivot check.
 * Dims: each odd and >= 3.  A level of odd dims coarsens to ((nx + 1) / 2, (ny + 1) / 2); the
 * first level with min(nx, ny) <= coarsest_n or an even dim is the coarsest, which must be at
 * most 65 points a side with at most 4096 unknowns (2^k + 1 dims reach 3; c 2^k + 1 with c
 * odd reaches c + 1).
 * Errors: DMG_ERR_DIMS, DMG_ERR_WORKSPACE, DMG_ERR_NOT_SPD, DMG_ERR_HIP. */
dmg_status dmg_workspace_bytes(int32_t nx, int32_t ny, const dmg_options* opts, size_t* bytes);
dmg_status dmg_setup(const double* S, int32_t nx, int32_t ny, const dmg_options* opts,
                     void* workspace, size_t ws_bytes, hipStream_t stream, dmg_hier** out);
void dmg_destroy(dmg_hier* h);
/* Recompute the whole hierarchy of h from a new fine stencil S of the same dims, in place (same
 * workspace, options and launch shapes).  Used when coefficients change (time stepping,
 * gradient steps: the hierarchy is recomputed rather than stored).  Asynchronous: the work is
 * enqueued on `stream` and the call returns without waiting (S must stay valid until that work
 * has run); a non-positive coarsest pivot (DMG_ERR_NOT_SPD) is reported by the next dmg_solve
 * on h.  From the second consecutive call with the same S pointer and stream (use_graph), the
 * setup is captured once into a hipGraph and replayed; it reads S's current contents. */
dmg_status dmg_refresh(dmg_hier* h, const double* S, hipStream_t stream);
/* dmg_assemble_stencil from (jac, K) followed by dmg_refresh, without the caller's stencil array:
 * the fine stencil is assembled straight into the hierarchy's level 0 (its planar and
 * point-major copies), then the coarse levels are recomputed.  The result equals that of
 * dmg_assemble_stencil into S followed by dmg_refresh(h, S) bit for bit (jac, K as
 * dmg_assemble_stencil takes them, for h's grid dims; they must stay valid until the work has
 * run).  Asynchronous like dmg_refresh; the graph is captured from the second consecutive call
 * with the same jac, K and stream. */
dmg_status dmg_refresh_assembled(dmg_hier* h, const double* jac, const double* K,
                                 hipStream_t stream);

/* Inspection of level l (0 = finest): dims and device pointers to its float64 stencil
 * [5][ny][nx] and (l < levels-1) interpolation weights [8][ny_c][nx_c] where entry (I,J) of
 * plane p holds: 0 w_W and 1 w_E of fine (2I+1,2J); 2 w_S and 3 w_N of fine (2I,2J+1);
 * 4..7 the weights of the centre fine point (2I+1,2J+1) to coarse (I,J),(I+1,J),(I,J+1),
 * (I+1,J+1).  Unused entries are 0. */
dmg_status dmg_hier_level(const dmg_hier* h, int32_t level, int32_t* nx, int32_t* ny,
                          const double** S, const double** P);
/* Levels, grid complexity sum N_l/N_1 and operator complexity sum nnz_l/nnz_1 (Sec. 4,
 * definitions of GC and OC; interior unknowns, stored 9-point nonzeros). Host-only. */
dmg_status dmg_stats(const dmg_hier* h, int32_t* levels, double* grid_complexity,
                     double* op_complexity);

/* ---- one V(nu_pre, nu_post) cycle on A u = b, in place on u (Sec. 2.2) -------------
 * Four-colour Gauss-Seidel smoothing, r = b - A u, b_H = P^T r, zero coarse initial guess,
 * recursion, coarsest Cholesky solve, u += P e_H, post-smoothing.  float64 only. */
dmg_status dmg_vcycle(dmg_hier* h, double* u, const double* b, hipStream_t stream);
/* One fused sweep kernel on `level` (float64), in the launch shape dmg_vcycle uses:
 * kind 0 = pre-smoothing sweep starting from u, followed by the restriction P^T (b - A u') into
 *          the next level's right-hand side;
 * kind 1 = post-smoothing sweep starting from u + P e (e = the next level's current
 *          correction).
 * The kernels work out of place: u is only read and the swept iterate u' goes to the level's
 * second iterate buffer inside the workspace.  u, b: [ny_l][nx_l] device arrays of that level.
 * level must be above the coarse tail (max(nx,ny) > 65); DMG_ERR_INVALID_ARG otherwise. */
dmg_status dmg_sweep(dmg_hier* h, int32_t level, int32_t kind, double* u, const double* b,
                     hipStream_t stream);
/* Autotuner.  flags bit 0: for every strip-kernel level pick the kernel and launch shape
 * (LDS strips of {64,128} columns, also 256 for float32, or one-wavefront strips that exchange
 * neighbour columns between lanes; segment height in {2,...,128} rows) with the lowest measured
 * time, for the pre and the post sweep separately: first each kernel alone (`reps` back-to-back
 * launches replayed from a captured graph and timed with hipEvents, so host launch overhead
 * does not enter), then level by level inside whole V-cycles (the faster of two graphs of
 * max(4, reps) cycles); float64 and, for DMG_FP32_IR, float32 kernels separately; and the coarse-tail
 * workgroup size -- launch shapes within one kernel family change no bit, a switch between
 * the LDS and the one-wavefront strip kernels only the rounding.  flags bit 1: pick the colour order with the
 * lowest measured solve time among the row-separable orders whose post order is the reverse of
 * the pre order (0123/3210, 1032/2301, 2301/1032, 3210/0123) -- this changes the iterates, so
 * read the choice back with dmg_hier_config.  flags bit 2 (DMG_FP32_IR): pick inner_cycles in
 * 1..8 with the lowest measured solve time to 1e-10 -- this changes the iterates (read it back
 * with dmg_hier_inner_cycles).  u is scratch (overwritten), b a right-hand side of the level-0
 * shape.  Synchronous.  Invalidates captured graphs. */
dmg_status dmg_autotune(dmg_hier* h, double* u, const double* b, int32_t flags, int32_t reps,
                        hipStream_t stream);
/* The launch shape of level `level`'s float64 pre sweep: bw = strip width in columns of the LDS
 * strip kernel, or 1 for the one-wavefront kernel; seg_h = rows per segment (0,0 for tail
 * levels); and the colour orders in use (host arrays of 4, nullable). */
dmg_status dmg_hier_config(const dmg_hier* h, int32_t level, int32_t* bw, int32_t* seg_h,
                           int32_t* pre_order, int32_t* post_order);
/* The float32 cycles per refinement step in use (dmg_options.inner_cycles, or the tuner's). */
dmg_status dmg_hier_inner_cycles(const dmg_hier* h, int32_t* inner_cycles);
/* The launch shape of level `level`'s float64 sweep of the given kind (0 pre, 1 post; the
 * autotuner picks them separately): bw and seg_h as in dmg_hier_config. */
dmg_status dmg_hier_sweep_config(const dmg_hier* h, int32_t level, int32_t kind, int32_t* bw,
                                 int32_t* seg_h);
/* ||b - A u||_2 over interior vertices (deterministic fixed-order reduction).  Synchronous. */
dmg_status dmg_residual_norm(dmg_hier* h, const double* u, const double* b, double* norm,
                             hipStream_t stream);
/* For callers that cannot allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc): the same residual norm without a hierarchy or workspace,
 * allocating nothing.  S [5][ny][nx] stencil, u, b [ny][nx] (device, caller-owned); norm (device,
 * caller-owned, 2 doubles) receives ||b - A u||_2^2 and ||b - A u||_2, bit for bit what
 * dmg_residual_norm computes on a hierarchy of S.  Asynchronous on `stream` (it does not
 * synchronise, so it can be captured).  The reduction partials live in one 8 KiB static device
 * array per device (kept until the process ends), fully rewritten by each call; its size does
 * not depend on the grid, so every grid with nx, ny >= 3 fits.  Calls that overlap on one device
 * (other streams, other host threads) share that array and race: serialise them.
 * Errors: DMG_ERR_INVALID_ARG, DMG_ERR_DIMS, DMG_ERR_HIP. */
dmg_status dmg_residual_norm_noalloc(const double* S, const double* u, const double* b,
                                     int32_t nx, int32_t ny, double* norm, hipStream_t stream);

/* ---- solve (Sec. 4 stopping rule: ||b - A u||_2 <= rtol ||b||_2) ------------------------
 * u in: initial guess, out: solution.  precision DMG_FP64: repeated V-cycles.  DMG_FP32_IR:
 * r = b - A x in fp64, s = ||r||_2 (on the device), r32 = fl32(r / s); inner_cycles fp32
 * V-cycles from e = 0 with fp32-rounded copies of the fp64 Galerkin stencils/weights (coarsest
 * solve in fp64); x += s e in fp64.  Dividing by ||r|| keeps r32 in float32's normal range
 * whatever the scale of b.  iters / relres (host,
 * nullable) return the count of cycles or refinement steps and the final relative residual;
 * history (host, nullable, >= max_iters doubles) receives the relative residual after each
 * step.  Returns DMG_ERR_NO_CONVERGENCE (u holds the last iterate) or DMG_ERR_NONFINITE.  The
 * convergence test runs on the device; the host synchronises `stream` after the start and the
 * first 4 steps, then after the steps the observed reduction per step predicts are left (at
 * most 16, enqueued as graphs of at most 4 steps).
 * The start tests u on the device: when every entry (boundary included) is zero, the initial
 * residual is b and is formed without a pass over the stencil, with the same bits. */
dmg_status dmg_solve(dmg_hier* h, double* u, const double* b, double rtol, int32_t max_iters,
                     int32_t* iters, double* relres, double* history, hipStream_t stream);

/* ---- per-cell gradient of J through the solve ---------------------------------------
 * dK[e] = -lambda_e^T G_e u_e, G_e the cell's Q1 element matrix (recomputed from jac as in
 * dmg_assemble_stencil), lambda and u vertex arrays with zero boundary ring.  With lambda
 * solving A lambda = dJ/du this is dJ/dK_e (discrete adjoint; A is symmetric). */
dmg_status dmg_grad_K(const double* jac, const double* lambda, const double* u, int32_t nx,
                      int32_t ny, double* dK, hipStream_t stream);

/* ---- grid <-> mesh transfers (Sec. 2.3 interpolation P = M_p^{-1} C, restriction P^T;
 * Sec. 2.3.1 coupled mass C) --------------------------------------------------------------
 * Two ways to create a transfer; the apply calls below work on either.
 *
 * From the caller's matrices (no allocation): C (Np x Nc) and M_p (Np x Np) as DEVICE CSR arrays,
 * int32 row pointers [Np + 1] starting at 0, int32 column indices and float64 values, borrowed:
 * they must stay valid and unchanged while the handle is used.  Columns of C index the grid
 * vector (vertex (i, j) of an nx x ny grid is column j nx + i, Nc = nx ny); Dirichlet treatment
 * (empty rows of C, identity rows of M_p) is the caller's.  The workspace (device, 256-byte
 * aligned, >= dmg_transfer_workspace_bytes for the same Np, Nc and nnz(C), owned by the caller
 * and outliving the handle) receives C^T, formed here on the device (rows in ascending mesh
 * order), and the CG vectors.  Create checks the CSR structure on the device (row pointers
 * non-decreasing, columns in range; DMG_ERR_INVALID_ARG otherwise) and synchronises `stream`.
 * Then from_grid = CG2(M_p, C u_c) and to_grid = C^T CG2(M_p, r_p) exactly as defined, with u_c
 * and r_c vectors of Nc entries and the mesh vectors in the caller's row order.
 * Errors: DMG_ERR_INVALID_ARG, DMG_ERR_WORKSPACE, DMG_ERR_HIP. */
dmg_status dmg_transfer_workspace_bytes(int32_t Np, int32_t Nc, int64_t nnz_C, size_t* bytes);
dmg_status dmg_transfer_create(int32_t Np, int32_t Nc, const int32_t* C_rowptr,
                               const int32_t* C_col, const double* C_val, const int32_t* M_rowptr,
                               const int32_t* M_col, const double* M_val, void* workspace,
                               size_t ws_bytes, hipStream_t stream, dmg_transfer** out);
/* From a P1 mesh given as HOST arrays (C and M_p assembled here): xy_c [nv][2] the images T(x_v) in (-1,1)^2,
 * xy_p [nv][2] physical coordinates, tris [nt][3] (int32, any orientation), dof [nv] (uint8,
 * 0 = Dirichlet vertex).  C is assembled by rasterising each mapped triangle over the grid
 * cells it overlaps with an nq x nq Gauss rule per cell, nq in [1, 32] (points outside the
 * triangle count as zero; |J_T^{-1}| taken as area(tau_p)/area(mapped tau)); nq = 0 integrates
 * exactly over each triangle-cell overlap polygon instead.  M_p is the P1 mass matrix.  The
 * handle owns device memory allocated here (freed by dmg_transfer_destroy); the apply calls
 * allocate nothing.  C and C^T are assembled on the device unless flags has
 * DMG_MESH_HOST_SETUP (or a row of C holds more than 64 grid columns, when the host assembly
 * takes over); both give the same bits.  M_p is assembled on the host (threads).
 * DMG_MESH_MATRIX_FREE (Sec. 2.3.1, closing remark; takes precedence over DMG_MESH_HOST_SETUP):
 * no C or C^T is stored.  Setup keeps the overlap sets -- per triangle its vertex images,
 * Jacobian factor and box of grid cells, per grid cell the triangles whose box holds it -- and
 * every apply recomputes the same triangle-cell integrals as the assembly (same nq rule), C u
 * by a gather per triangle then per mesh row, C^T y by a gather per grid cell then per grid
 * vertex, in fixed orders (deterministic; equal to the assembled form's results to rounding).
 * Device memory drops from two CSR copies of C to 16 B per vertex + ~20 B per triangle + 4 B per
 * triangle-cell pair + a buffer of max(3 nt, 4 cells) float64; each apply costs the integrals
 * once more.  dmg_transfer_copy_C then returns DMG_ERR_UNSUPPORTED and nnz_C reads 0.
 * from_grid: u_p = CG2(M_p, C u_c)      u_c [ny][nx] -> u_p [nv]
 * to_grid:   r_c = C^T CG2(M_p, r_p)    r_p [nv]     -> r_c [ny][nx]
 * CG2 = two iterations of unpreconditioned CG from 0.  Dirichlet entries are ignored/zero. */
dmg_status dmg_transfer_create_mesh(int32_t nv, int32_t nt, const double* xy_c,
                                    const double* xy_p, const int32_t* tris, const uint8_t* dof,
                                    int32_t nx, int32_t ny, int32_t nq, int32_t flags,
                                    hipStream_t stream, dmg_transfer** out);
dmg_status dmg_transfer_info(const dmg_transfer* t, int64_t* nnz_C, int64_t* nnz_M);
/* Device bytes that hold C (its CSR and C^T's, or the matrix-free overlap sets with their buffer)
 * and the triangle-cell pairs of the overlap sets (0 unless matrix-free); nullable outputs. */
dmg_status dmg_transfer_memory(const dmg_transfer* t, size_t* bytes_C, int64_t* overlap_pairs);
/* C as a host CSR with rows in the caller's vertex order: rp [nv + 1], ci and v [nnz_C] (from
 * dmg_transfer_info), columns ascending within a row.  Synchronous. */
dmg_status dmg_transfer_copy_C(const dmg_transfer* t, int32_t* rp, int32_t* ci, double* v);
dmg_status dmg_transfer_from_grid(dmg_transfer* t, const double* u_c, double* u_p,
                                  hipStream_t stream);
dmg_status dmg_transfer_to_grid(dmg_transfer* t, const double* r_p, double* r_c,
                                hipStream_t stream);
void dmg_transfer_destroy(dmg_transfer* t);

/* ---- batched solve of independent instances ----------------------------------------
 * count instances with dims nx[k], ny[k] (host arrays, any mix of sizes dmg_setup accepts) and fine stencils
 * S[k] (host array of device pointers).  One workspace holds every hierarchy plus the batch's
 * schedule.  dmg_batch_solve runs one batched V-cycle per step: each fused sweep is launched
 * once per level size over the tiles of every instance having a level of that size (largest
 * first going down, smallest first going up), then every instance's coarse tail (one workgroup
 * each) and convergence check.  Four steps are captured in one hipGraph (when `stream` is not
 * the legacy default stream) and replayed until each instance meets ||b - A u|| <= rtol ||b||
 * or max_iters; a converged instance's work stops at once.  The iterates equal those of
 * dmg_solve on each instance.  u (in: initial guess, out: solution) and b are host arrays of
 * device pointers; iters / relres (host, [count], nullable) receive per-instance counts and
 * final relative residuals.  float64 only (DMG_ERR_UNSUPPORTED otherwise); with point smoothing
 * nu_pre + nu_post must be even.  With line relaxation (opts.smoother 1-3) each level size runs
 * its unfused line steps (coarse start, sweeps, residual, restriction, interpolation) as one
 * launch each over its instances, and the iterates equal dmg_solve's with coarse_gemv = 0.
 * Returns DMG_ERR_NO_CONVERGENCE if any instance did not converge. */
dmg_status dmg_batch_workspace_bytes(int32_t count, const int32_t* nx, const int32_t* ny,
                                     const dmg_options* opts, size_t* bytes);
dmg_status dmg_batch_setup(int32_t count, const int32_t* nx, const int32_t* ny,
                           const double* const* S, const dmg_options* opts, void* workspace,
                           size_t ws_bytes, hipStream_t stream, dmg_batch** out);
dmg_status dmg_batch_solve(dmg_batch* bt, double* const* u, const double* const* b,
                           double rtol, int32_t max_iters, int32_t* iters, double* relres,
                           hipStream_t stream);
/* Batch autotuner, synchronous; u is scratch (overwritten), b the right-hand sides.
 * flags bit 0: the wave-strip segment height of each level size and the coarse-tail workgroup
 * size, by timing `reps` batched steps each -- numerically neutral.
 * flags bit 1 (point smoothing only; ignored with line relaxation, which visits no colours):
 * the colour-order pair (the same four row-separable pairs as dmg_autotune, post order the
 * reverse of the pre order) of each size class (the instances with one finest grid size), class
 * by class, by timing whole batched solves to 1e-10 from zero; each instance's dense coarse
 * operators are rebuilt for its pair.  This changes the iterates: read the choices back with
 * dmg_batch_instance_orders.  Bit 1 runs first. */
dmg_status dmg_batch_autotune(dmg_batch* bt, double* const* u, const double* const* b,
                              int32_t flags, int32_t reps, hipStream_t stream);
/* Instance 0's colour orders (host arrays of 4, nullable) and the coarse-tail workgroup size. */
dmg_status dmg_batch_config(const dmg_batch* bt, int32_t* pre_order, int32_t* post_order,
                            int32_t* tail_threads);
/* Instance k's colour orders (host arrays of 4, nullable). */
dmg_status dmg_batch_instance_orders(const dmg_batch* bt, int32_t k, int32_t* pre_order,
                                     int32_t* post_order);
void dmg_batch_destroy(dmg_batch* bt);

/* ---- the two-level cycle on the physical mesh (Sec. 2.2, solution phase) -----------------
 * Solves A_p u_p = f_p, A_p the P1 stiffness of the physical mesh (element matrices K_t G_t on
 * the physical triangles, Dirichlet rows and columns replaced by the identity), with stationary
 * cycles: a symmetric multicolour Gauss-Seidel sweep, r_c = C^T M^{-1} (f_p - A_p u_p), one
 * float64 V-cycle of `grid` on A_c e_c = r_c from e_c = 0, u_p += M^{-1} C e_c, a second
 * symmetric sweep.  M^{-1} is mass = 0: the lumped mass (row sums of M_p), or mass = 2: two CG
 * iterations on M_p (Sec. 2.3).  Colours: greedy on the mesh graph (unknowns sharing a
 * triangle are neighbours; Dirichlet vertices have none, colour 0) with the vertices in
 * smallest-last order (each removed in turn as one of least degree among those left, the
 * smallest index among equals; coloured in reverse removal order); the symmetric sweep updates
 * colours 0..C-1 then C-2..0.
 * Create: mesh arrays on the HOST, nq and flags as for dmg_transfer_create_mesh (nq = 0, the exact overlap
 * integral, keeps the coarse correction's energy matched to A_p as the mesh is refined; low
 * quadrature orders let it drift); K_t [nt] host coefficient per
 * triangle (null: 1); grid: a hierarchy built on the nx x ny grid that C maps to (its level-0
 * dims), borrowed -- it must outlive the handle, and no other call may use it while a cycle or
 * solve of this handle runs.  The handle owns device memory allocated here; cycle and solve
 * allocate nothing.  DMG_ERR_INVALID_ARG for a degenerate physical triangle or a non-positive
 * diagonal of A_p.
 * info: number of colours, stored entries of A_p (nullable outputs); colour (nullable, host
 * [nv]) receives each vertex's colour.
 * cycle: one cycle on u_p [nv] (device, in/out) for f_p [nv] (device).
 * solve: cycles from u_p until ||f - A u|| <= rtol ||f - A u_0|| or max_iters; a zero initial
 * residual returns at once with iters = 0 and relres = 0.  history (host, nullable,
 * >= max_iters entries) receives ||f - A u_k|| / ||f - A u_0||.  Chunks of at most four cycles
 * run in one captured hipGraph each (when `stream` is not the legacy default stream); the host
 * synchronises after the first chunk, then after the cycles the observed reduction per cycle
 * predicts are left (at most 16, as back-to-back chunks).  Returns
 * DMG_ERR_NO_CONVERGENCE or DMG_ERR_NONFINITE with u_p holding the last iterate. */
dmg_status dmg_twolevel_create(int32_t nv, int32_t nt, const double* xy_c, const double* xy_p,
                               const int32_t* tris, const uint8_t* dof, const double* K_t,
                               dmg_hier* grid, int32_t nq, int32_t mass, int32_t flags,
                               hipStream_t stream, dmg_twolevel** out);
dmg_status dmg_twolevel_info(const dmg_twolevel* tl, int32_t* colours, int64_t* nnz_A,
                             int32_t* colour);
dmg_status dmg_twolevel_cycle(dmg_twolevel* tl, double* u_p, const double* f_p,
                              hipStream_t stream);
dmg_status dmg_twolevel_solve(dmg_twolevel* tl, double* u_p, const double* f_p, double rtol,
                              int32_t max_iters, int32_t* iters, double* relres, double* history,
                              hipStream_t stream);
/* Coarse-grid scaling (Sec. 2.4): set_scaling makes later cycles add gamma P e_c (default 1;
 * any finite value).  scaling estimates gamma as the mean of the Ritz values of k steps
 * (k in [1, 64]; the paper's k = 12) of the generalized Lanczos recurrence for
 * P^T A_p P x = lambda A_c x in the A_c-inner product, i.e. trace(T_k) / k, started from the
 * interior part of v0 (device [ny][nx], caller-chosen, e.g. seeded uniform values).  Each step
 * applies P^T A_p P once and solves with A_c by the grid hierarchy's float64 solve (relative
 * residual 1e-13); the recurrence stops early when the Krylov space is invariant
 * (beta_j <= 1e-13 |alpha_j|).  gamma (host) receives the estimate, steps (nullable) the steps
 * taken m, T (host, nullable, [k][k]) the m x m tridiagonal in its leading block, zeros
 * elsewhere.  The estimate does not change the handle's gamma.  Lumped mass only
 * (DMG_ERR_UNSUPPORTED for CG2, whose P is not linear).  Synchronous; allocates nothing (its
 * six grid vectors of scratch are part of a lumped-mass handle from creation). */
dmg_status dmg_twolevel_set_scaling(dmg_twolevel* tl, double gamma);
dmg_status dmg_twolevel_scaling(dmg_twolevel* tl, const double* v0, int32_t k, double* gamma,
                                double* T, int32_t* steps, hipStream_t stream);
void dmg_twolevel_destroy(dmg_twolevel* tl);

#ifdef __cplusplus
}
#endif
#endif /* DMG_H */
