// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/afdcg.h"

namespace afd {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
struct Status {
    int code = AFD_OK;
};
#define AFD_HIP_TRY(expr)                                                          \
    do {                                                                           \
        hipError_t _e = (expr);                                                    \
        if (_e != hipSuccess) {                                                    \
            ::afd::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));   \
            return AFD_E_HIP;                                                      \
        }                                                                          \
    } while (0)
#define AFD_TRY(expr)                   \
    do {                                \
        int _s = (expr);                \
        if (_s != AFD_OK) return _s;    \
    } while (0)

// AFD_OK or AFD_E_INVALID_ARG (with the message set) for a mesh description
int validate_desc(const afd_mesh_desc& d);
// the mesh's context, the context's stream and the mesh description
afd_context* mesh_context(const afd_mesh* m);
hipStream_t context_stream(const afd_context* c);
const afd_mesh_desc& mesh_desc(const afd_mesh* m);
int mesh_dof_mask(const afd_mesh* m, uint8_t* host);  // the fixity per DOF, copied to the host

// ------------------------------------------------------------ element data
// The element matrix in the tensor-product Haar basis.  Per axis, a node pair
// (v0, v1) maps to (s, d) = (v0 + v1, v1 - v0); in that basis the isotropic
// voxel matrix is block-sparse: a diagonal dg[i][alpha] (alpha = 3-bit Haar
// index, bit k = difference along axis k) and, for i != j, a coupling of
// (alpha, i) with (alpha ^ e_i ^ e_j, j) whose value depends only on the
// third axis k and its bit: lam*Mk/4 when alpha_i = 1, mu*Mk/4 when
// alpha_j = 1 (Mk = hk/4 for bit 0, hk/12 for bit 1).
struct KeHaar {
    double dg[3][8];      // dg[i][alpha]; dg[i][0] = 0 (translations)
    double cl[3][2];      // lam * M_k(bit) / 4, indexed [k][bit_k]
    double cm[3][2];      // mu  * M_k(bit) / 4
    double kdiag[3];      // diagonal of Ke for component c
};
KeHaar make_ke_haar(const double h[3], double E, double nu);
void make_ke_dense(const double h[3], double E, double nu, double* ke576);  // row-major, LOCAL order

// -------------------------------------------------------------- geometry
struct Grid {
    int nx, ny, nz;          // elements per axis
    int64_t nnode, nelem, ndof;
};

// Deflation block geometry
struct Blocks {
    int b[3];                // block edge (elements)
    int nb[3];               // blocks per axis
    int nblk;                // total blocks
    int ncoarse;             // 6 * nblk
    double inv_scale;        // 1 / max(b)
    int perm[3];             // axis order of the coarse ordering (fastest first)
    int P;                   // super-block size of the block-tridiagonal coarse matrix
    int K;                   // number of super-blocks
    int w;                   // half bandwidth in the permuted ordering
    int m;                   // middle super-block of the two-ended order, (K - 1) / 2
};

// Two-ended order of the super-blocks of the banded coarse matrix: the first
// m keep their place and orientation (chain A, positions 0..m-1), the last
// K-1-m follow in reverse order with their unknowns reversed (chain B,
// positions m..K-2; reversing a banded matrix keeps it banded, so B is block
// tridiagonal with the same coupling windows as A), and super-block m,
// reversed, goes last (position K-1), coupled to both chain ends.  The
// factorisation and both triangular solves then run the two chains side by
// side toward or away from the middle: about K/2 dependent steps instead of
// K - 1.  Position of banded index q:
inline int twist_position(int q, int P, int K, int m) {
    const int j = q / P, r = q - j * P;
    if (j < m) return q;
    if (j == m) return (K - 1) * P + (P - 1 - r);
    return (m + K - 1 - j) * P + (P - 1 - r);
}

// Super-block size of the block-tridiagonal coarse factor: any multiple of 64
// that is >= the half bandwidth w is valid.  A coarse solve (two-ended order,
// see twist_position) is 2 floor((K-2)/2) + 5 dependent launches: the paired
// chain steps (P x w matrix-vector products; the coupling blocks are zero
// outside a w-column window), one launch for the middle block each way, the
// permutation and two batched passes over the K triangular inverses (K P^2 / 2
// entries each).  Cost model fitted to measured solves on MI355X: ~6 us per
// dependent launch plus the streamed bytes at ~4.5 TB/s.  Pick the P of least
// modelled time among w, 2w, ..., 6w (AFD_COARSE_P overrides).
inline int choose_coarse_P(int ncoarse, int w) {
    const int nc64 = ((ncoarse + 63) / 64) * 64;
    int forced = 0;
    if (const char* e = getenv("AFD_COARSE_P")) forced = atoi(e);
    if (forced > 0) {
        int P = ((std::max(forced, w) + 63) / 64) * 64;
        return std::min(P, nc64);
    }
    const double lat = 6e-6, bw = 4.5e12;
    int best = 0;
    double best_t = 1e30;
    for (int m = 1; m <= 6; ++m) {
        int P = ((m * w + 63) / 64) * 64;
        if (P > nc64) P = nc64;
        const int K = (ncoarse + P - 1) / P;
        const double bytes = 2.0 * (K - 1) * P * std::min(P, w) * 8.0 + 2.0 * K * (double)P * P * 4.0;
        const double t = (K >= 2 ? 2.0 * ((K - 2) / 2) + 5.0 : 3.0) * lat + bytes / bw;
        if (t < best_t - 1e-12) {
            best_t = t;
            best = P;
        }
        if (P == nc64) break;
    }
    return best;
}

// Device memory of the library.  Every allocation and free goes through
// these, under one process-wide lock that the recording of an iteration graph
// (stream capture and instantiation) also holds: hipFree synchronises the
// device, and no allocation or free of one thread (a server slot creating or
// dropping a mesh) may overlap a capture in another (a slot recording its
// iterations), nor may two captures overlap.  Replays need no lock.
std::recursive_mutex& device_memory_mutex();
hipError_t dev_malloc_raw(void** p, size_t bytes);
hipError_t dev_free(void* p);
template <typename T>
inline hipError_t dev_malloc(T** p, size_t bytes) {
    return dev_malloc_raw(reinterpret_cast<void**>(p), bytes);
}

// Per-right-hand-side CG scalars, device resident.
struct CgScalars {
    double rz, rz_new, pq, alpha, beta, rr, bb, rr0;
    double tol2;             // (rtol * ||b||)^2 threshold on r.r
    int32_t done;            // 0 running, 1 converged, 2 breakdown, 3 max_iter
    int32_t iters;
    int32_t max_iter;
    int32_t xdone;           // the direction kernel has applied the x update of the iteration that set done
};

// persist.hip: the FP64 deflated PCG as one launch, one workgroup per
// right-hand side (see afd_mesh_solver_form)
constexpr int64_t PERSISTENT_MAX_ELEMS = 65536;  // largest mesh of the form
bool persistent_fits(const Grid& g, const Blocks& b, bool deflate, int nrhs);
int launch_dcg_persistent(const Grid& g, const Blocks& b, bool deflate, const KeHaar& kh, const double* rho,
                          const uint8_t* nmask, const double* rinv, const double* Linv, const double* LinvT,
                          const int32_t* perm, const int32_t* iperm, int nrhs, const double* F, double* X, double* R,
                          double* P, double* Q, double* Z, double* Ye, CgScalars* sc, double rtol, int max_iter,
                          bool warm, hipStream_t s);

// --------------------------------------------------------------- launchers
// matvec.hip
struct MatvecArgs {
    Grid g;
    const double* rho;       // nelem
    const float* rho32;      // nelem (FP32 path)
    const uint8_t* nmask;    // nnode, bit c = DOF c fixed
    const double* rho_t;     // tile-major densities (plain apply), see launch_tile_rho
    const float* rho32_t;
    const uint16_t* fm_t;    // tile-major face fixity words, see launch_tile_fmask
    int apply_variant[2] = {-1, -1};  // plain-apply kernel per precision (FP64, FP32), -1 default
    int apply_zc[2] = {0, 0};         // plain-apply z chunk per precision, 0 default
};
struct DcgArgs {
    const double* rinv;      // nnode: 1 / sum of rho over the node's elements
    CgScalars* sc;           // [nrhs]
    double* partial;         // [(rhs*2 + which) * npart + i]
    int npart;
};
int matvec_num_tiles(const Grid& g);
// element counts of the tile-major side arrays of the plain apply: returns the
// fixity-word count, *nrho the density count
int64_t tile_layout_sizes(const Grid& g, int64_t* nrho);
// default z chunk of a plain-apply kernel variant for nrhs right-hand sides
// (zc_req > 0 forces it)
void apply_tiling(const Grid& g, int fp32, int variant, int zc_req, int nrhs, int* zc, int* nchunk);
int launch_tile_rho(const Grid& g, const double* rho, double* rho_t, float* rho32_t, hipStream_t s);
int launch_tile_fmask(const Grid& g, const uint8_t* nmask, uint16_t* fm_t, hipStream_t s);
// p' = beta p + M^-1 r - W mu (MU null: no deflation), zero on fixed DOFs
// X (may be null): also x += alpha p_old, the x update of the iteration
// (k_cg_update then runs without X)
int launch_form_dir(const Grid& g, const Blocks& b, const uint8_t* nmask, const KeHaar& kh, const CgScalars* sc,
                    int nrhs, const double* MU, const double* rinv, const double* Pold, const double* R,
                    double* Pnew, double* X, hipStream_t s);
int launch_form_dir_f32(const Grid& g, const Blocks& b, const uint8_t* nmask, const KeHaar& kh,
                        const CgScalars* sc, int nrhs, const double* MU, const float* rinv32, const float* Pold,
                        const float* R, float* Pnew, float* X, hipStream_t s);
// Q = A P with the per-workgroup partial sums of P.Q (d.partial, slot 0 of
// each right-hand side), skipping converged right-hand sides (d.sc)
int launch_apply_dot(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, int fp32, int nrhs, const void* P,
                     void* Q, hipStream_t s);
int launch_apply(const MatvecArgs& a, const KeHaar& kh, int fp32, int nrhs, const void* U, void* Y,
                 hipStream_t s);
int launch_residual(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, int nrhs, const double* F,
                    const double* X, double* R, hipStream_t s);
int launch_residual_f32(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, const float* rinv32, int nrhs,
                        const float* F, const float* X, float* R, hipStream_t s);
int launch_apply_mfma(const MatvecArgs& a, const double* ke576_dev, int nrhs, const double* U, double* Y,
                      hipStream_t s);

// vec.hip
constexpr int VEC_NPART = 1024;
int launch_pack_mask(const Grid& g, const uint8_t* dofmask, uint8_t* nmask, hipStream_t s);
int launch_node_rsum(const Grid& g, const double* rho, double* rinv, float* rinv32, hipStream_t s);
int launch_jacobi_full(const Grid& g, const double* rinv, const uint8_t* nmask, const KeHaar& kh, double* d,
                       hipStream_t s);
int launch_dot(int64_t n, const double* x, const double* y, double* partial, int npart, double* out,
               hipStream_t s);
int launch_dot_rhs(int64_t ndof, int nrhs, const double* F, double* partial, int npart, hipStream_t s);
int launch_dot_rhs_f32(int64_t ndof, int nrhs, const float* F, double* partial, int npart, hipStream_t s);
int launch_cg_init(CgScalars* sc, int nrhs, const double* part, int npart, double rtol, int max_iter,
                   hipStream_t s);
int launch_cg_start(CgScalars* sc, int nrhs, const double* part, int npart, hipStream_t s);
int launch_scalar_beta(CgScalars* sc, int nrhs, const double* part, int npart, hipStream_t s);
// alpha from the p.q partials (pqpart, npq per right-hand side, as the
// direction apply writes them), then the r/z update with its r.z and r.r
// partials; X, Pv may be null: no x update (the deflated PCG does it in
// launch_form_dir)
int launch_cg_update(const Grid& g, const KeHaar& kh, const double* rinv, CgScalars* sc, int nrhs, double* X,
                     const double* Pv, double* R, const double* Q, double* Z, double* partial, int npart,
                     const double* pqpart, int npq, hipStream_t s);
int launch_cg_update_f32(const Grid& g, const KeHaar& kh, const float* rinv32, CgScalars* sc, int nrhs, float* X,
                         const float* Pv, float* R, const float* Q, float* Z, double* partial, int npart,
                         const double* pqpart, int npq, hipStream_t s);
int launch_precond(const Grid& g, const KeHaar& kh, const double* rinv, int nrhs, const double* R, double* Z,
                   hipStream_t s);
int launch_precond_f32(const Grid& g, const KeHaar& kh, const float* rinv32, int nrhs, const float* R, float* Z,
                       hipStream_t s);
int launch_restrict(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* V, double* G,
                    hipStream_t s);
// G = W^T (V - V2); optionally also gperm[r][perm[i]] = G[r][i] (npad per
// right-hand side: the coarse solve's permuted input, see coarse_solve) and
// the CG beta/convergence update of sc from bpart (k_scalar_beta's work)
int launch_restrict_diff(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* V,
                         const double* V2, double* G, hipStream_t s, const int32_t* perm = nullptr,
                         double* gperm = nullptr, int64_t npad = 0, CgScalars* sc = nullptr,
                         const double* bpart = nullptr, int bnpart = 0);
int launch_restrict_diff_f32(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const float* V,
                             const float* V2, double* G, hipStream_t s, const int32_t* perm = nullptr,
                             double* gperm = nullptr, int64_t npad = 0, CgScalars* sc = nullptr,
                             const double* bpart = nullptr, int bnpart = 0);
int launch_restrict_f32(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const float* V, double* G,
                        hipStream_t s);
int launch_prolong(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* MU, double* V,
                   hipStream_t s);
// X[r] += W MU[r] on free DOFs and X[r] = 0 on fixed DOFs (MU null: masking
// only); X[r] = 0 where sc[r].done (sc may be null)
int launch_prolong_add(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* MU,
                       const CgScalars* sc, double* X, hipStream_t s);
int launch_prolong_f32(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* MU, float* V,
                       hipStream_t s);
int launch_probe_vector(const Grid& g, const Blocks& b, const uint8_t* nmask, int color, int mode, double* V,
                        hipStream_t s);
int launch_copy_f64(int64_t n, const double* a, double* b, hipStream_t s);
int launch_fill_f64(int64_t n, double v, double* a, hipStream_t s);
int launch_fill_f32(int64_t n, float v, float* a, hipStream_t s);
// mixed precision helpers
int launch_to_f32_scaled(int64_t ndof, int nrhs, const double* R, const CgScalars* outer, float* Rf, hipStream_t s);
int launch_axpy_refine(int64_t ndof, int nrhs, const CgScalars* outer, const float* D, double* X, hipStream_t s);
int launch_outer_norm(CgScalars* outer, int nrhs, const double* part, int npart, hipStream_t s);

// dense.hip : coarse matrix and its block Cholesky
struct Coarse {
    Blocks blk;
    double* D = nullptr;     // K x P x P : diagonal blocks of E, then L_kk
    double* B = nullptr;     // K x P x P : sub-diagonal blocks E_{k+1,k}, then C_k = L_{k+1,k}
    double* Linv = nullptr;  // K x P x P : L_kk^-1
    double* LinvT = nullptr; // K x P x P : (L_kk^-1)^T
    double* T = nullptr;     // K x P x P : T_k = Linv_k C_{k-1}
    double* U = nullptr;     // K x P x P : U_k = Linv_k^T C_k^T
    double* Ediag = nullptr; // K*P original diagonal
    double* work = nullptr;  // P x P
    double* work2 = nullptr; // P x P, for the second chain of the factorisation
    hipStream_t s2 = nullptr;                        // second chain's stream
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int32_t* dropped_dev = nullptr;
    int32_t* perm = nullptr; // natural coarse index -> ordered index
    int32_t* iperm = nullptr; // ordered index -> natural coarse index (-1: padding), K*P
    std::vector<int32_t> iperm_host;  // staging of iperm (lives until the copy has run)
    double* gperm = nullptr; // [4][K*P]
    double* xperm = nullptr; // [4][K*P]
    // FP32 copies of Linv, LinvT, T and U for the FP32 inner solves of the
    // mixed form (made on demand after a factorisation; FP64 accumulation)
    float* Linv32 = nullptr;
    float* LinvT32 = nullptr;
    float* T32 = nullptr;
    float* U32 = nullptr;
    int dropped = 0;
    bool valid = false;
    bool valid32 = false;
};
int coarse_alloc(Coarse& c, hipStream_t s);
void coarse_free(Coarse& c);
int coarse_begin(Coarse& c, hipStream_t s);
int coarse_scatter_probe(Coarse& c, const double* G, int color, int mode, hipStream_t s);
// E = W^T A W directly from the element matrices (after coarse_begin); rigid:
// equal voxel edges, so elements inside one block with no fixed DOF add nothing
int coarse_direct(Coarse& c, const Grid& g, const double* rho, const uint8_t* nmask, const double* ke576,
                  bool rigid, hipStream_t s);
int coarse_factor(Coarse& c, hipStream_t s);
int coarse_make_f32(Coarse& c, hipStream_t s);  // FP32 copies of the solve matrices (after coarse_factor)
// mu = E^-1 g; f32: stream the FP32 copies (requires valid32), vectors and accumulation stay FP64
// g_in_perm: G's permuted copy is already in c.gperm (written by the
// restriction), so the permutation launch is skipped
int coarse_solve(Coarse& c, int nrhs, const double* G, double* MU, hipStream_t s, bool f32 = false,
                 bool g_in_perm = false);
int coarse_to_dense_host(Coarse& c, double* E_host, hipStream_t s);  // before factor only

// post.hip
int launch_sensitivity(const Grid& g, const KeHaar& kh, const double* rho, int nfields, const double* const* Ua,
                       const double* const* Ub, double* S, hipStream_t s);
// casting projection of an element field on a dims grid (see afd_casting)
int launch_cast(const int dims[3], int axis, int parting, const double* phi, double* out, hipStream_t s);
int launch_parting_distance(const int dims[3], int axis, int parting, int32_t* dist, hipStream_t s);
// out = sum_t coef[t] * (sum of the rows[t] rows of fields[t]), left to right, no FMA (t < 4)
int launch_combine(int64_t n, int nterms, const double* const* fields, const int* rows, const double* coef,
                   double* out, hipStream_t s);
// p-norm von Mises stress of nrhs displacement fields (see afd_stress_pnorm)
int stress_pnorm(const Grid& g, const double h[3], double E, double nu, const double* rho, const uint8_t* nmask,
                 int nrhs, const double* U, double p, double* vm, double* pn_host, double* B, hipStream_t st);
// modal.hip: consistent mass apply and the subspace-iteration eigen-solver (see afd_apply_M, afd_modal)
int mass_apply(const Grid& g, const double h[3], const double* rho, const uint8_t* nmask, int nrhs, const double* U,
               double* Y, hipStream_t s);
// the subspace block of the eigen-solver between runs: 4 columns of n_dof
// (device, owned by the caller), their Ritz values mu = 1 / lambda, and
// whether they hold a run's result
struct EigenBlock {
    double* X = nullptr;
    double mu[4] = {0.0, 0.0, 0.0, 0.0};
    bool valid = false;
};
int modal_subspace(afd_mesh* mesh, const Grid& g, const double h[3], const double* rho, const uint8_t* nmask,
                   const afd_solve_opts* inner, int nev, double tol, int max_iter, double* lam_out, double* Phi,
                   double* S, afd_modal_stats* st, hipStream_t s, EigenBlock* block = nullptr);
// afd_modal with a start block (see EigenBlock), for the optimisation loop
int modal_with_block(afd_mesh* m, const afd_solve_opts* inner, int nev, double tol, int max_iter, double* lam,
                     double* Phi, double* S, afd_modal_stats* st, EigenBlock* block);
// geometric stiffness of the centroid stresses of U0 (see afd_apply_Kg, afd_buckling)
int geo_apply(const Grid& g, const double h[3], double E, double nu, const double* rho, const uint8_t* nmask,
              const double* U0, int nrhs, const double* X, double* Y, hipStream_t s);
int buckling_subspace(afd_mesh* mesh, const Grid& g, const double h[3], double E, double nu, const double* rho,
                      const uint8_t* nmask, const double* U, const afd_solve_opts* inner, int nev, double tol,
                      int max_iter, double* lam_out, double* Phi, double* S, afd_modal_stats* st, hipStream_t s,
                      EigenBlock* block = nullptr);
// afd_buckling with a start block (see EigenBlock), for the optimisation loop
int buckling_with_block(afd_mesh* m, const double* U, const afd_solve_opts* inner, int nev, double tol, int max_iter,
                        double* lam, double* Phi, double* S, afd_modal_stats* st, EigenBlock* block);
// rho[e] = solid[e] ? 1 : void_scale
int launch_density(int64_t n, const uint8_t* solid, double void_scale, double* rho, hipStream_t s);
// ranking and threshold (see afd_threshold): threshold_run on a caller-given
// device work space of threshold_work_bytes(n); threshold_gpu allocates it
size_t threshold_work_bytes(int64_t n);
int threshold_run(const double* s, const int32_t* tie, int64_t n, double vol_frac, uint8_t* solid, int32_t* order,
                  double* tau_host, void* work, hipStream_t st);
int threshold_gpu(const double* s, const int32_t* tie, int64_t n, double vol_frac, uint8_t* solid, int32_t* order,
                  double* tau_host, hipStream_t st);
// the allocation-free form: the work space is a static device array of
// THRESHOLD_NOALLOC_BYTES (threshold_work_bytes(AFD_THRESHOLD_NOALLOC_MAX))
// whose per-device address threshold_scratch_init takes (device current)
constexpr size_t THRESHOLD_NOALLOC_BYTES = 51381248;
int threshold_scratch_init(int device);
int threshold_noalloc(int device, const double* s, const int32_t* tie, int64_t n, double vol_frac, uint8_t* solid,
                      int32_t* order, double* tau_host, hipStream_t st);

}  // namespace afd
