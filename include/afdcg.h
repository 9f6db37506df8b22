/*
 * afdcg.h - C ABI of the MI355X assembly-free deflated voxel solver.
 *
 * The library solves the linear static problem K u = f of a finite element
 * model (Eq. 1.1 of Deng & Suresh, "Multi-Constrained 3D Topology Optimization
 * Via Augmented Topological Level-Set") on a box of nx*ny*nz voxels meshed by
 * 8-node hexahedra (Sec. 3.8, step 1), with an assembly-free deflated
 * conjugate gradient (Sec. 3.5), and returns the compliance J = f.u
 * (Eq. 1.3-1.4), per-element strain-energy sensitivity fields (the element
 * term u^T K^e u of Eq. 3.5, Sec. 3.1) and the topology extracted from such a
 * field at a volume fraction (Eq. 3.6, Sec. 3.2).
 *
 * Conventions used by every call:
 *   element e = ex + nx*(ey + ny*ez); node n = i + (nx+1)*(j + (ny+1)*k);
 *   DOF 3*n + c (c = x, y, z): displacement-type vectors are interleaved per
 *   node; a block of nrhs vectors is stored row-major [nrhs][ndof].
 *   Element e has stiffness rho_e * Ke, Ke the 24x24 matrix of an isotropic
 *   hx*hy*hz voxel (E, nu).  A DOF flagged fixed is a homogeneous Dirichlet
 *   DOF: the solver works with the operator A = K_ff on free DOFs, extended by
 *   the identity on fixed DOFs (so A is SPD on the whole DOF vector).
 *
 * Pointers: unless a call says otherwise, array arguments are DEVICE
 * pointers on the context's device and kernels run asynchronously on the
 * context's stream; calls named "host" take host pointers and return after
 * the data has been copied.  The caller owns every buffer it passes.
 *
 * Errors: every call returns an int status (AFD_OK = 0, negative on error);
 * afd_last_error() gives a thread-local message for the last failure on the
 * calling thread.  No exception crosses this boundary.  Objects are not
 * thread-safe, except the server.
 */
#ifndef AFDCG_H
#define AFDCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define AFD_OK                 0
#define AFD_PENDING            1   /* server: request not finished yet          */
#define AFD_E_INVALID_ARG     -1   /* bad size, pointer, value or state          */
#define AFD_E_NO_DEVICE       -2   /* no HIP device / bad device index           */
#define AFD_E_OOM             -3   /* device allocation failed                   */
#define AFD_E_OVER_BUDGET     -4   /* request larger than the server budget      */
#define AFD_E_NOT_CONVERGED   -5   /* max_iter reached; outputs hold last iterate */
#define AFD_E_BREAKDOWN       -6   /* p.Ap <= 0 or non-finite (singular K)       */
#define AFD_E_COARSE_SINGULAR -7   /* every coarse pivot dropped                 */
#define AFD_E_HIP             -8   /* a HIP runtime call failed                  */

#define AFD_MEM_HOST   0
#define AFD_MEM_DEVICE 1

#define AFD_FP64  0   /* FP64 throughout                                         */
#define AFD_MIXED 1   /* FP32 inner deflated PCG under FP64 iterative refinement */
#define AFD_FP32  2   /* afd_apply_K, autotuner: FP32 vectors and arithmetic;     *
                       * afd_mesh_coarse_precision: FP32 coarse solve matrices   */

typedef struct afd_context afd_context;
typedef struct afd_mesh afd_mesh;
typedef struct afd_server afd_server;

/* Geometry/material of a voxel mesh (Sec. 3.8 step 1: hexahedral elements;
 * Sec. 4 states the material as E and nu).  bx,by,bz: edge (in elements) of
 * the agglomerated element blocks whose six rigid-body motions span the
 * deflation space of Sec. 3.5; 0 in any of them disables deflation. */
typedef struct {
    int32_t nx, ny, nz;
    double hx, hy, hz;
    double E, nu;
    int32_t bx, by, bz;
} afd_mesh_desc;

typedef struct {
    double rtol;          /* stop when ||f - A u||_2 <= rtol * ||f||_2            */
    int32_t max_iter;     /* CG iterations (FP64) or inner iterations per sweep   */
    int32_t precision;    /* AFD_FP64 or AFD_MIXED                               */
    double inner_rtol;    /* MIXED: residual reduction of the first inner solve;
                             later sweeps reduce by what is still missing to rtol
                             (x1/2 margin), within [max(inner_rtol/100, 1e-6), 1/2] */
    int32_t check_every;  /* iterations between host convergence checks (>=1)    */
    int32_t mem_kind;     /* AFD_MEM_HOST or AFD_MEM_DEVICE for F, U, J, S       */
    const int32_t* pairs; /* host array of 2*npairs RHS indices (a,b)            */
    int32_t npairs;       /* mutual-energy fields requested                      */
    int32_t max_refine;   /* MIXED: outer refinement sweeps (<=0: 30)            */
    const double* x0;     /* start, nrhs x n_dof (host or device per mem_kind;
                             values on fixed DOFs are ignored) or NULL: the
                             deflated start W E^-1 W^T f.  FP64 starts from
                             x0 + W E^-1 W^T (f - A x0); MIXED refines from x0.
                             A warm start from a nearby solution (Sec. 3.2: the
                             fixed-point loop re-solves after small topology
                             changes) needs few iterations                      */
} afd_solve_opts;

typedef struct {
    int32_t iterations;       /* total CG iterations (inner, for MIXED)           */
    int32_t refinements;      /* MIXED: outer sweeps; FP64: restarts on the true
                                 residual                                         */
    int32_t status;           /* AFD_OK or the failure of this right-hand side    */
    int32_t coarse_dropped;   /* coarse columns dropped as rank-deficient         */
    double rel_residual_true; /* ||f - A u|| / ||f|| recomputed in FP64 at exit    */
    double t_setup, t_iter, t_post; /* seconds (host wall clock, stream-synced)   */
} afd_solve_stats;

/* ---- context ----------------------------------------------------------- */
/* Opens device `device`.  `hip_stream` is a hipStream_t to run on (e.g.
 * torch.cuda.current_stream().cuda_stream) or NULL for a library-owned stream.
 * AFD_E_NO_DEVICE if the device does not exist. */
int afd_context_create(int device, void* hip_stream, afd_context** out);
void afd_context_destroy(afd_context* ctx);
/* Message of the last failure on the calling thread ("" if none). */
const char* afd_last_error(void);
/* Blocks until the context's stream is idle. */
int afd_context_sync(afd_context* ctx);
/* Solver iterations between host convergence checks (check_every, when even)
 * are recorded once per mesh as a HIP graph and replayed (default on); 0
 * launches them one by one instead.  Results are identical either way.
 * Recording is a stream capture: no other thread may make device-synchronising
 * HIP calls (hipMalloc, hipFree, synchronous copies) on the device meanwhile,
 * so turn it off for contexts that solve while other threads allocate (the
 * server's slot contexts have it off). */
int afd_context_use_graphs(afd_context* ctx, int32_t enable);

/* ---- mesh -------------------------------------------------------------- */
/* Creates the device-resident state of a voxel mesh (no stiffness matrix is
 * ever assembled: Sec. 3.5).  All rho start at 1 and no DOF is fixed.
 * AFD_E_INVALID_ARG for n* < 1, h* <= 0, E <= 0, nu outside (-1, 0.5), b* < 0. */
int afd_mesh_create(afd_context* ctx, const afd_mesh_desc* desc, afd_mesh** out);
void afd_mesh_destroy(afd_mesh* mesh);
/* Sizes: number of elements, nodes, DOFs, coarse unknowns (6 per block). */
int afd_mesh_sizes(const afd_mesh* mesh, int64_t* n_elem, int64_t* n_node,
                   int64_t* n_dof, int64_t* n_coarse);

/* Per-element stiffness scale rho_e (> 0, finite), n_elem values, host or
 * device per mem_kind; copied (stream-ordered).  Invalidates the Jacobi
 * diagonal and the coarse factor (rebuilt at the next use).  Host input is
 * validated (AFD_E_INVALID_ARG on a non-positive or non-finite value). */
int afd_mesh_set_scale(afd_mesh* mesh, const double* rho, int64_t n_elem, int mem_kind);
/* Fixity: one uint8 per DOF, nonzero = fixed (homogeneous Dirichlet). */
int afd_mesh_set_fixed(afd_mesh* mesh, const uint8_t* dof_mask, int64_t n_dof, int mem_kind);
/* Device bytes a solve of nrhs right-hand sides at `precision` will hold
 * (mesh state + coarse factor + Krylov work space): used for admission. */
int afd_mesh_footprint(const afd_mesh* mesh, int32_t nrhs, int32_t precision, uint64_t* bytes);

/* ---- hot-path steps (device pointers, asynchronous on the context stream) */
/* The element matrix Ke (24x24 row-major, local node order bottom face
 * counter-clockwise then top face, DOF 3a+c) as the library uses it,
 * written to a HOST buffer of 576 doubles.  (K^e of Eq. 3.5.) */
int afd_mesh_ke(const afd_mesh* mesh, double* ke_host);

/* Element-by-element operator apply (the assembly-free K.u of Sec. 3.5):
 * Y[r] = A U[r] for r < nrhs, A = sum_e rho_e P_e^T Ke P_e restricted to free
 * DOFs, identity on fixed DOFs.  precision AFD_FP64 (double U, Y) or
 * AFD_FP32 (float U, Y).  U and Y must not overlap.  nrhs in 1..4. */
int afd_apply_K(afd_mesh* mesh, int32_t precision, int32_t nrhs, const void* U, void* Y);
/* Multi-RHS apply with the dense 24x24 Ke x [U_e...] contraction on the
 * FP64 matrix cores (same result as afd_apply_K, FP64 only, nrhs 1..4). */
int afd_apply_K_mfma(afd_mesh* mesh, int32_t nrhs, const double* U, double* Y);

/* Autotuner of afd_apply_K for this mesh (the operator of Sec. 3.5 is fixed;
 * only its execution is tuned): times every candidate kernel variant x z
 * chunking of the element-by-element apply for `precision` (AFD_FP64 or
 * AFD_FP32) and `nrhs` on the context stream with HIP events, and keeps the
 * fastest (if it beats the default by 3% or more) for later afd_apply_K calls
 * on this mesh with that precision
 * (every candidate evaluates the same element operator; results agree to
 * rounding).  Synchronous; allocates and frees two scratch vectors of
 * nrhs x n_dof.  report may be NULL. */
typedef struct afd_tune_report {
    int32_t variant;        /* chosen kernel: 0 register-staged, 2 / 3 LDS-DMA with 1 / 2 layers per step,
                               4 / 6 buffer-load LDS-DMA with a prefetch distance of 2 / 1 layers,
                               -1 the default (variant 6; kept unless a candidate is >= 3% faster) */
    int32_t zc;             /* chosen node planes per z chunk                                           */
    double us;              /* its time per launch (microseconds)                                       */
    double default_us;      /* time of the untuned default                                              */
    int32_t ncandidates;    /* candidates timed                                                         */
} afd_tune_report;
int afd_mesh_autotune(afd_mesh* mesh, int32_t precision, int32_t nrhs, afd_tune_report* report);
/* Sets the afd_apply_K execution for `precision` by hand (what the autotuner
 * picks): variant 0 register-staged, 2 / 3 LDS-DMA with 1 / 2 layers per
 * step, 4 / 6 buffer-load LDS-DMA with a prefetch distance of 2 / 1 layers,
 * -1 the default; zc node planes per z chunk, 0 the default.  Returns
 * AFD_E_INVALID_ARG for other values. */
int afd_mesh_apply_config(afd_mesh* mesh, int32_t precision, int32_t variant, int32_t zc);
/* Element type of the coarse solve matrices the deflated iterations of
 * afd_solve stream (Sec. 3.5's coarse problem W^T K W, always factored in
 * FP64): AFD_FP64 streams the FP64 factor; AFD_FP32 uses FP32 copies made
 * once per factorisation, with FP64 vectors and accumulation (half the bytes
 * per coarse solve; the coarse correction is then exact to ~1e-7 relative,
 * the stopping test and the true residual stay FP64).  By default (no call)
 * the FP64 iterations stream the FP64 factor (the copies if the environment
 * sets AFD_COARSE_F32=1) and the FP32 inner solves of AFD_MIXED stream the
 * copies; AFD_FP64 set here makes both stream the factor, AFD_FP32 both the
 * copies.  AFD_E_INVALID_ARG otherwise. */
int afd_mesh_coarse_precision(afd_mesh* mesh, int32_t precision);
/* Execution form of the FP64 deflated PCG of afd_solve on this mesh (the
 * iteration of Sec. 3.5 is the same in both forms, only its execution
 * differs):
 *   AFD_FORM_LAUNCHES   (the default) a chain of launches per iteration,
 *                       recorded as HIP graphs in chunks of check_every
 *                       iterations;
 *   AFD_FORM_PERSISTENT one launch for the whole solve, one workgroup of 1024
 *                       threads per right-hand side iterating until its
 *                       stopping test, on one compute unit per right-hand
 *                       side (for meshes of at most 65,536 elements whose
 *                       coarse problem fits one super-block of at most 1024
 *                       unknowns; afd_solve returns AFD_E_INVALID_ARG for a
 *                       larger one).  Slower per solve than the chain at every
 *                       size measured; it leaves the rest of the chip to
 *                       concurrent work.
 * The mixed form always runs the launch chain.  AFD_E_INVALID_ARG for other
 * values. */
#define AFD_FORM_LAUNCHES   0
#define AFD_FORM_PERSISTENT 1
int afd_mesh_solver_form(afd_mesh* mesh, int32_t form);

/* Jacobi diagonal of A (Sec. 3.5: preconditioner formed assembly-free):
 * d[3n+c] = Ke_cc * sum of rho over the elements touching node n for a free
 * DOF, 1 for a fixed DOF.  d: ndof doubles. */
int afd_jacobi(afd_mesh* mesh, double* d);

/* Deterministic FP64 dot product of two length-n device vectors; the result
 * is written to *out_dev (device).  Fixed-order reduction: bitwise
 * reproducible run to run. */
int afd_dot(afd_context* ctx, int64_t n, const double* x, const double* y, double* out_dev);

/* Deflation operators (W: six rigid motions per block, zero on fixed DOFs).
 * Coarse vectors are [nrhs][n_coarse], entry 6*b + m for block
 * b = bi + nbx*(bj + nby*bk) and motion m in (tx, ty, tz, rx, ry, rz); the
 * motions are taken about the centre of the block's node range, in element
 * units divided by max(bx,by,bz).  Node i (per axis) belongs to block
 * min(i / b, nb - 1), nb = ceil(n_elem_axis / b). */
int afd_restrict(afd_mesh* mesh, int32_t nrhs, const double* V, double* G);   /* G = W^T V */
int afd_prolong(afd_mesh* mesh, int32_t nrhs, const double* MU, double* V);   /* V = W MU  */
/* Builds E = W^T A W without assembling A and factors it by block Cholesky
 * (done lazily by afd_solve; this call forces it).  Returns the number of
 * coarse columns dropped as rank-deficient in *dropped (may be NULL).
 * E is summed from the element matrices of the elements along block
 * interfaces (and of those with fixed DOFs; of every element when the voxel
 * edges differ), in a fixed order, so it is bit-reproducible; with the
 * environment variable AFD_COARSE_ASSEMBLY=probe it is built instead from
 * 162 operator applies of 3x3x3-coloured motion probes (Sec. 3.5). */
int afd_coarse_setup(afd_mesh* mesh, int32_t* dropped);
/* E as a dense HOST matrix n_coarse x n_coarse (row-major), for checking;
 * only for n_coarse <= 8192. */
int afd_coarse_matrix(afd_mesh* mesh, double* E_host);
/* MU = E^-1 G (dropped columns give 0), nrhs in 1..4. */
int afd_coarse_solve(afd_mesh* mesh, int32_t nrhs, const double* G, double* MU);

/* Per-element energies: S[f][e] = rho_e u_e^T Ke v_e, f < nrhs + npairs:
 * fields 0..nrhs-1 pair U[f] with itself (strain energy, sum_e = f.u = J);
 * field nrhs+p pairs U[pairs[2p]] with U[pairs[2p+1]] (mutual energy).
 * pairs is a HOST array.  (Element term of Eq. 3.5.) */
int afd_sensitivity(afd_mesh* mesh, int32_t nrhs, const double* U,
                    int32_t npairs, const int32_t* pairs, double* S);

/* Topology at volume fraction vol_frac in [0,1] (Eq. 3.6, Sec. 3.2): the
 * ceil(vol_frac*n) elements first in the order (s descending, index
 * ascending) are solid (solid[e] = 1, else 0); *tau_host receives s of the
 * last solid element (+inf if none).  Values compare as numbers (-0.0 ranks
 * as +0.0).  tie (optional, may be NULL): an int32 key >= 0 per element that
 * ranks equal values before the index, order (s descending, tie ascending,
 * index ascending) -- for a field from afd_casting pass its dist output, so
 * that plateaus are cut nearer the parting plane first and the topology has
 * no cavity (Sec. 3.7).  order (optional, may be NULL) receives the full
 * ranking as int32 element indices.  s, tie, solid, order: device.
 * Synchronous (returns after the ranking); allocates a work space of ~24 B
 * per element for the call. */
int afd_threshold(afd_context* ctx, const double* s, const int32_t* tie, int64_t n, double vol_frac,
                  uint8_t* solid, int32_t* order, double* tau_host);

/* afd_threshold for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, results and synchronisation, but the ranking's work space
 * is a static device array of the library (49 MiB, held on every GPU the
 * library runs on until the process ends), so the call makes no hipMalloc,
 * hipFree or other allocating call.  n must be <= AFD_THRESHOLD_NOALLOC_MAX
 * (AFD_E_INVALID_ARG otherwise).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (two threads, or streams of two contexts)
 * race and must be serialised by the caller. */
#define AFD_THRESHOLD_NOALLOC_MAX 2097152
int afd_threshold_noalloc(afd_context* ctx, const double* s, const int32_t* tie, int64_t n, double vol_frac,
                          uint8_t* solid, int32_t* order, double* tau_host);

/* Casting constraint (Sec. 3.7): out = the least element field >= phi that
 * does not increase away from the parting plane along the casting axis, so
 * that a topology extracted from it (afd_threshold with dist as the tie key)
 * has no cavity a mould drawn along the axis cannot reach.  dims = elements
 * per axis (x fastest: element ex + dims[0] (ey + dims[1] ez)); axis 0, 1 or
 * 2; the parting plane lies before element index parting along the axis
 * (0..dims[axis]; 0 or dims[axis]: one-sided casting).  Along every line of
 * elements parallel to the axis this is the running maximum from each far
 * end toward the plane.  phi and out are device arrays of
 * dims[0]*dims[1]*dims[2] doubles (finite values); out may equal phi.  Exact
 * (maxima only; a zero is written as +0.0).  dist (optional device int32
 * array of the same size, may be NULL) receives each element's distance from
 * the plane in elements along the axis (j - parting on the side j >= parting,
 * parting - 1 - j before it).  AFD_E_INVALID_ARG for a bad axis, dims or
 * parting. */
int afd_casting(afd_context* ctx, const int32_t dims[3], const double* phi, int32_t axis, int32_t parting,
                double* out, int32_t* dist);

/* p-norm von Mises stress (the stress constraint of Eq. 3.21 / 3.23 and the
 * adjoint field of Eq. 3.3) of nrhs (1..4) displacement fields U (device,
 * [nrhs][n_dof]) on the mesh's current densities: element stresses at the
 * voxel centre sigma_e = rho_e D B_c u_e, von Mises vm_e, and
 * *pn_host = (sum_r sum_e vm_{e,r}^p)^(1/p) over every element and field
 * (p >= 2, e.g. 8).  vm (optional device [nrhs][n_elem]) receives vm_e.  B
 * (optional device [nrhs][n_dof]) receives the adjoint right-hand sides
 * d pn / d U[r] = pn^(1-p) sum_e vm_e^(p-2) rho_e B_c^T D V sigma_e (V the
 * von Mises quadratic form), zero on fixed DOFs: afd_solve of B gives the
 * adjoint fields lambda_r, and the mutual energies of (U[r], lambda_r)
 * (afd_sensitivity pairs) are the stress sensitivity field.  Synchronous;
 * allocates a work space of up to 48 B per element per field. */
int afd_stress_pnorm(afd_mesh* mesh, int32_t nrhs, const double* U, double p, double* vm, double* pn_host,
                     double* B);

/* ---- modal analysis (the eigenvalue constraint of Eq. 3.21; Eq. 3.4) ----- */
/* Y[r] = M U[r] for r < nrhs (1..4): the consistent mass matrix of the voxel
 * (unit density, int N^T N per component), each element's mass scaled by its
 * stiffness scale rho_e, applied element by element on the free DOFs (fixed
 * inputs taken as zero, 0 on fixed DOFs).  U, Y: device, FP64, [nrhs][n_dof]. */
int afd_apply_M(afd_mesh* mesh, int32_t nrhs, const double* U, double* Y);

typedef struct {
    int32_t iterations;        /* subspace iterations                            */
    int32_t cg_iterations;     /* CG iterations of all the inner solves          */
    int32_t converged;         /* 1 when every Ritz residual met tol             */
    double rel_residual[3];    /* ||K phi - lambda M phi|| / (lambda ||M phi||)  */
    double t;                  /* seconds                                        */
} afd_modal_stats;
/* The nev (1..3) lowest eigenpairs of K phi = lambda M phi on the free DOFs
 * (the free vibration problem whose lowest eigenvalue Eq. 3.21 constrains)
 * by subspace iteration on a block of 4 vectors: each iteration one 4-column
 * deflated solve K Y = M X (afd_solve with *inner's rtol and precision,
 * warm-started from X / lambda) and a Rayleigh-Ritz projection, until every
 * reported pair's Ritz residual is <= tol (AFD_E_NOT_CONVERGED after max_iter
 * iterations; the outputs then hold the last Ritz pairs).  lambda_host: nev
 * eigenvalues ascending; Phi: device [nev][n_dof], M-normalised (phi^T M phi
 * = 1), sign arbitrary; S (optional device [nev][n_elem]): the eigenvalue
 * sensitivity field of each pair, rho_e phi_e^T (K_e - lambda M_e) phi_e
 * (Eq. 3.4 by the element route).  Synchronous; allocates 4 x 4 work vectors. */
int afd_modal(afd_mesh* mesh, const afd_solve_opts* inner, int32_t nev, double tol, int32_t max_iter,
              double* lambda_host, double* Phi, double* S, afd_modal_stats* stats);

/* ---- linear buckling (Eq. 3.5; the buckling constraints of Eq. 3.21, 3.24) */
/* Y[r] = K_sigma X[r] for r < nrhs (1..4): the geometric stiffness of the
 * stress state of the displacement field U0 (device, one field), each
 * element's stress taken at its centre (rho_e D B_c u_e, as in
 * afd_stress_pnorm): K_sigma,e[(a,i),(b,j)] = delta_ij sum_pq S_pq
 * int dN_a/dx_p dN_b/dx_q; elements whose scale rho_e is below 1/2 (the
 * ersatz void) carry no stress and add nothing (their scaled stress over
 * their soft strains would give spurious local modes near zero load); on the
 * free DOFs (fixed inputs taken as zero, 0 on fixed DOFs).  Synchronous;
 * allocates 48 B per element for the call. */
int afd_apply_Kg(afd_mesh* mesh, const double* U0, int32_t nrhs, const double* X, double* Y);
/* The nev (1..3) smallest positive load factors lambda of
 * (K + lambda K_sigma) phi = 0 for the stress state of U (device, the static
 * solution under the applied loads; the critical load is lambda times them),
 * by the subspace iteration of afd_modal on -K_sigma x = mu K x (largest mu,
 * lambda = 1 / mu).  Phi: device [nev][n_dof], phi^T K phi = 1; S (optional
 * device [nev][n_elem]): the load-factor sensitivity field of Eq. 3.5 by the
 * element route with the prebuckling stresses held,
 * lambda phi_e^T (rho_e K_e + lambda K_sigma,e) phi_e.  stats as afd_modal
 * (residual ||K phi + lambda K_sigma phi|| / ||K phi||).  AFD_E_BREAKDOWN if
 * fewer than nev positive load factors are found. */
int afd_buckling(afd_mesh* mesh, const double* U, const afd_solve_opts* inner, int32_t nev, double tol,
                 int32_t max_iter, double* lambda_host, double* Phi, double* S, afd_modal_stats* stats);

/* The augmented topological level set (Eq. 3.17-3.18): out[e] =
 * sum_t coef[t] * (sum_{r < rows[t]} fields[t][r * n + e]), terms and rows
 * added left to right without fused multiply-adds (so it is the double the
 * plain expression gives).  fields: HOST array of nterms (1..4) DEVICE
 * pointers, group t holding rows[t] fields of n values (e.g. the strain
 * energies of the load cases: their sum is the compliance sensitivity);
 * rows, coef: HOST.  out: device, n doubles. */
int afd_combine_fields(afd_context* ctx, int64_t n, int32_t nterms, const double* const* fields,
                       const int32_t* rows, const double* coef, double* out);

/* ---- the whole solve ---------------------------------------------------- */
/* Solves A U[r] = F[r] for r < nrhs (1..4) by deflated Jacobi-PCG (Sec. 3.5),
 * FP64 or FP32-inner/FP64-refined per opts->precision (the coarse factor is
 * computed in FP64 and applied through FP32 copies where
 * afd_mesh_coarse_precision says so; the stopping test and the reported true
 * residual are FP64),
 * then writes the compliances J[r] = F[r].U[r] (Eq. 1.3) and, if S != NULL,
 * the energy fields of afd_sensitivity (opts->pairs).  F, U, J, S are host or device per
 * opts->mem_kind.  F must be zero on fixed DOFs (AFD_E_INVALID_ARG
 * otherwise when F is on the host).  stats (host, may be NULL) receives nrhs
 * records.  A column succeeds when the true FP64 residual of the returned
 * U[r], ||F[r] - A U[r]|| / ||F[r]|| recomputed at exit, is <= rtol: the FP64
 * iteration stops on its recursive residual at 0.99 rtol and restarts from
 * its iterate (up to 3 times) while the true residual is above rtol; the
 * mixed form refines on the true residual.  Returns AFD_OK when every column
 * succeeded, else the first failing column's status: AFD_E_NOT_CONVERGED when
 * max_iter, the restarts or the refinement sweeps ran out above rtol (a target
 * below the FP64 attainable accuracy of the problem ends so), AFD_E_BREAKDOWN;
 * U then holds the last iterate. */
int afd_solve(afd_mesh* mesh, const afd_solve_opts* opts, int32_t nrhs,
              const double* F, double* U, double* J, double* S, afd_solve_stats* stats);

/* ---- the optimisation loop (Sec. 3.2-3.4, 3.6, 3.8; Fig. 6-7) ------------ */
/* Pareto tracing of minimum volume from the full design domain downward
 * under the hard constraint J <= alpha_J J0 (Eq. 3.21-3.22; J the sum of the
 * load cases' compliances, J0 its value on the full domain) and optionally
 * sigma_PN <= alpha_sigma sigma_PN0 (Eq. 3.23, afd_stress_pnorm; its adjoint
 * solve per step, g_s, mu_s, gamma_s by the same rules, and the term
 * w_s T_sigma / (alpha_sigma sigma_PN0) of the level set, T_sigma the mutual
 * energies of the load cases and their adjoint fields).  Per solve k:
 * the finite element solves of every load case (afd_solve, warm-started from
 * the previous displacements), g = J / (alpha_J J0) - 1, the multiplier and
 * penalty updates mu <- max(mu + gamma g, 0) and Eq. 3.12 (gamma kept at
 * k = 0), then
 *  - g > 0 (hard constraint violated), or max_fp solves at one target
 *    without convergence: back to the last converged feasible design
 *    (volume v_b), dv halved, next target v_b - dv (stop when dv < dv_min);
 *  - else the augmented level set T_L = w T_J / (alpha_J J0),
 *    w = max(mu + gamma g, 0) (1 when 0), T_J the sum of the element
 *    strain-energy fields; converged when the compliance moved by less than
 *    conv_tol since the previous solve at the same target (the full domain
 *    counts as converged), and then the target drops by dv (stop at <= 0);
 *  - the next topology: the ceil(v nE) elements of highest T_L (with the
 *    casting constraint, Sec. 3.7: of the projected field, ties cut nearer
 *    the parting plane first), void elements at void_scale.
 * With alpha_lambda > 0 the lowest eigenvalue joins as a hard constraint
 * lambda_1 >= alpha_lambda lambda_10 (Eq. 3.21; afd_modal on each topology,
 * void elements scaled in mass as in stiffness): g_l = 1 - lambda_1 /
 * (alpha_lambda lambda_10), its own mu_l, gamma_l by the same rules, and the
 * term w_l T_lambda / (alpha_lambda lambda_10) of the level set, T_lambda the
 * eigenvalue field of afd_modal (Eq. 3.4: the drop of lambda_1 when an
 * element loses stiffness and mass); with lambda_soft it is a soft
 * constraint (Sec. 3.6, Eq. 3.20-3.21): its violation does not count as one.
 * With alpha_P > 0 the smallest buckling load factor P of load case 0's
 * stress state joins the same way (afd_buckling on each topology):
 * P >= alpha_P P_0, g_p = 1 - P / (alpha_P P_0), mu_p, gamma_p, the term
 * w_p T_P / (alpha_P P_0) with T_P the load-factor field of afd_buckling;
 * P_soft makes it soft.  The eigen-solves of each step start from the Ritz
 * block of the previous step and run at most 200 subspace iterations; one
 * that does not meet modal_tol ends the loop with its status.
 * With damping the topology is extracted from the mean of the solve's level
 * set and the level set its topology was extracted from (a fixed point that
 * would alternate between two topologies settles).
 * The mesh's fixity is used and its densities are overwritten (on return
 * they are those of the last solved topology).  F: HOST, nload (1..4) x n_dof,
 * zero on fixed DOFs.  solid: HOST, n_elem, receives the last converged
 * feasible design.  hist: HOST, hist_cap records (*n_hist receives the count;
 * the loop also stops after hist_cap or max_fea solves); topo_hist: HOST,
 * optional (NULL), hist_cap x n_elem, receives the topology of every solve.
 * Returns AFD_OK when the loop ended by its rules or its solve budget, else
 * the failing call's status (the history up to it is kept).  Allocates its
 * device work space for the call. */
#define AFD_LS_FIXED_POINT 0   /* another fixed-point solve at the same target    */
#define AFD_LS_CONVERGED   1   /* converged (and feasible): the target drops by dv */
#define AFD_LS_VIOLATED    2   /* hard constraint violated: dv halved, step back   */
#define AFD_LS_DIVERGED    3   /* no convergence within max_fp: as a violation     */
#define AFD_LS_TERMINATED  4   /* the loop ended after this solve                  */
typedef struct {
    double alpha_J;            /* >= 1                                          */
    double dv0, dv_min;        /* Sec. 4.2: 0.025; stop below dv_min             */
    double mu0, gamma0;        /* Sec. 3.8 step 1: 100, 10                       */
    double varsigma, eta;      /* Eq. 3.12: 0.25, 10                             */
    double conv_tol;           /* step 7: 0.01                                   */
    int32_t max_fp, max_fea;   /* solves per target before a divergence; total   */
    double void_scale;         /* ersatz scale of void elements (e.g. 1e-3)      */
    int32_t cast_axis;         /* casting constraint: 0..2, or -1 for none       */
    int32_t cast_parting;      /* parting plane index along cast_axis            */
    double alpha_sigma;        /* stress constraint sigma_PN <= alpha_sigma
                                  sigma_PN0 (Eq. 3.23), <= 0: none; needs
                                  nload <= 2                                     */
    double pnorm_p;            /* p of the stress p-norm (>= 2, e.g. 8)          */
    int32_t damping;           /* 1: extract from the mean of the solve's level
                                  set and the one its topology came from         */
    afd_solve_opts solve;      /* the solves (mem_kind, pairs, x0 are set by the loop) */
    double alpha_lambda;       /* eigenvalue constraint lambda_1 >= alpha_lambda
                                  lambda_10, 0 < alpha_lambda <= 1; <= 0: none   */
    double modal_tol;          /* Ritz residual of the eigenpair (e.g. 1e-9); its
                                  inner solves take the rtol of `solve`          */
    int32_t lambda_soft;       /* 1: the eigenvalue constraint is soft (Sec. 3.6):
                                  its term shapes the level set, its violation
                                  neither steps back nor ends the loop          */
    double alpha_P;            /* buckling constraint P >= alpha_P P_0 (load case
                                  0), 0 < alpha_P <= 1; <= 0: none              */
    int32_t P_soft;            /* 1: the buckling constraint is soft            */
} afd_levelset_opts;
typedef struct {
    int32_t fea;               /* solve index                                    */
    int32_t event;             /* AFD_LS_*                                       */
    int32_t nsolid;            /* solid elements of the solved topology          */
    int32_t iterations;        /* CG iterations of the solves (summed over loads,
                                  adjoint solves and eigen-solves)              */
    double v;                  /* target volume fraction of the solved topology  */
    double J, g;               /* compliance and constraint value               */
    double mu, gamma;          /* after this solve's update                      */
    double dv;                 /* volume step after this solve's decision        */
    double t_fea, t_total;     /* seconds: this solve (afd_solve, all load
                                  cases) and the whole step (solve, fields,
                                  level set, extraction, bookkeeping)           */
    double S, g_s, mu_s, gamma_s; /* stress p-norm, its constraint value, its
                                  multiplier and penalty (0 without it)         */
    double lam, g_l, mu_l, gamma_l; /* lowest eigenvalue, its constraint value,
                                  multiplier and penalty (0 without it)         */
    double P, g_p, mu_p, gamma_p; /* smallest buckling load factor, its
                                  constraint value, multiplier and penalty     */
} afd_levelset_record;
int afd_levelset_run(afd_mesh* mesh, const afd_levelset_opts* opts, int32_t nload, const double* F,
                     uint8_t* solid, afd_levelset_record* hist, int32_t hist_cap, int32_t* n_hist,
                     uint8_t* topo_hist);

/* ---- serving ------------------------------------------------------------ */
typedef struct {
    afd_mesh_desc desc;
    const double* rho;        /* host, n_elem              */
    const uint8_t* fixed;     /* host, n_dof               */
    const double* F;          /* host, nrhs * n_dof        */
    int32_t nrhs;
    afd_solve_opts opts;      /* mem_kind ignored (host); pairs and x0 (host) copied */
} afd_request;

typedef struct {
    double* U;                /* host, nrhs * n_dof, caller-owned (may be NULL) */
    double* J;                /* host, nrhs (may be NULL)                        */
    afd_solve_stats* stats;   /* host, nrhs (may be NULL)                        */
    int32_t status;           /* filled on completion                            */
    double t_submit, t_start, t_done; /* seconds on the server's clock           */
} afd_result;

/* Continuous-batching solve server on one device: requests are admitted as
 * slots and HBM budget free up, run concurrently on per-slot streams, and
 * complete independently.  hbm_budget in bytes (0 = 90% of free memory). */
int afd_server_create(afd_context* ctx, uint64_t hbm_budget, int32_t max_slots, afd_server** out);
/* Copies the request (the caller may free it on return); `res` must stay
 * valid until the ticket completes.  Thread-safe. */
int afd_server_submit(afd_server* srv, const afd_request* req, afd_result* res, uint64_t* ticket);
/* AFD_PENDING while running, else the request's final status. */
int afd_server_poll(afd_server* srv, uint64_t ticket);
/* Waits up to timeout_s (<0: forever); AFD_PENDING on timeout. */
int afd_server_wait(afd_server* srv, uint64_t ticket, double timeout_s);
/* Server clock now (seconds). */
double afd_server_clock(afd_server* srv);
/* Finishes queued work, then frees everything. */
void afd_server_destroy(afd_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* AFDCG_H */
