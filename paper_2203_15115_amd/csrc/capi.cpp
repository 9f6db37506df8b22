// C ABI and host runtime: context and mesh state, the deflated PCG driver
// (Sec. 3.5), FP32-inner / FP64-refined mixed precision, compliance
// (Eq. 1.3) and element energies (Eq. 3.5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "afd_internal.h"

namespace afd {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static bool verbose() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("AFD_VERBOSE");
        v = (e && *e && *e != '0') ? 1 : 0;
    }
    return v == 1;
}

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int validate_desc(const afd_mesh_desc& d) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1 || !(d.hx > 0) || !(d.hy > 0) || !(d.hz > 0) || !(d.E > 0) ||
        !(d.nu > -1.0 && d.nu < 0.5) || d.bx < 0 || d.by < 0 || d.bz < 0 || !std::isfinite(d.hx) ||
        !std::isfinite(d.hy) || !std::isfinite(d.hz) || !std::isfinite(d.E)) {
        set_error("invalid mesh description (need n >= 1, h > 0, E > 0, -1 < nu < 0.5, b >= 0)");
        return AFD_E_INVALID_ARG;
    }
    const int64_t nnode = (int64_t)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    if (3 * nnode >= ((int64_t)1 << 31)) {
        set_error("mesh too large (3 * nodes must fit in int32)");
        return AFD_E_INVALID_ARG;
    }
    return AFD_OK;
}

std::recursive_mutex& device_memory_mutex() {
    static std::recursive_mutex mu;
    return mu;
}
hipError_t dev_malloc_raw(void** p, size_t bytes) {
    std::lock_guard<std::recursive_mutex> lk(device_memory_mutex());
    return hipMalloc(p, bytes);
}
hipError_t dev_free(void* p) {
    std::lock_guard<std::recursive_mutex> lk(device_memory_mutex());
    return hipFree(p);
}

}  // namespace afd

using namespace afd;

struct afd_context {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool graphs = true;         // replay recorded solver iteration chunks
    double* scratch = nullptr;  // dot partials
};

struct Work {
    int nrhs = 0;
    int mixed = 0;
    // FP64 Krylov state [nrhs][ndof]
    double *X = nullptr, *R = nullptr, *P0 = nullptr, *P1 = nullptr, *Q = nullptr, *Z = nullptr, *AZ = nullptr;
    double *F = nullptr;   // device copy of F (host input)
    double* Ye = nullptr;  // persistent form: per-element outputs of the apply [nrhs][24][nelem]
    double *S = nullptr;   // energies (host output)
    // FP32 inner state
    float *Xf = nullptr, *Rf = nullptr, *P0f = nullptr, *P1f = nullptr, *Qf = nullptr, *Zf = nullptr,
          *AZf = nullptr, *Bf = nullptr;
    double *G = nullptr, *MU = nullptr;  // coarse vectors [4][ncoarse]
    CgScalars* sc = nullptr;             // [4] inner / FP64
    CgScalars* outer = nullptr;          // [4] refinement
    double *partM = nullptr, *partV = nullptr;
    double* Jdev = nullptr;
};

// one recorded chunk of solver iterations and what was baked into it
struct IterGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> key;
    void release() {
        std::lock_guard<std::recursive_mutex> lk(afd::device_memory_mutex());
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        key.clear();
    }
};

struct afd_mesh {
    afd_context* ctx = nullptr;
    afd_mesh_desc desc{};
    Grid g{};
    KeHaar kh{};
    Blocks blk{};
    int deflate = 0;
    double* rho = nullptr;
    float* rho32 = nullptr;
    uint8_t* nmask = nullptr;
    uint8_t* dofmask = nullptr;  // staging for set_fixed
    double* rho_t = nullptr;     // tile-major copies for the plain apply
    float* rho32_t = nullptr;
    uint16_t* fm_t = nullptr;
    double* rinv = nullptr;
    float* rinv32 = nullptr;
    double* ke_dev = nullptr;    // dense Ke (576) for the matrix-core path
    bool jacobi_valid = false;
    bool any_fixed = false;
    IterGraph graphs[2];             // recorded iteration chunks (FP64 solve, FP32 inner solve)
    int coarse_f32 = -1;             // coarse solve matrices streamed in FP32 (1) or FP64 (0); -1: default
    int tune_variant[2] = {-1, -1};  // autotuned plain-apply kernel per precision (FP64, FP32)
    int tune_zc[2] = {0, 0};
    int solver_form = AFD_FORM_LAUNCHES;
    Coarse coarse;
    Work w;
    int npartM = 0;
};

namespace afd {
afd_context* mesh_context(const afd_mesh* m) { return m->ctx; }
hipStream_t context_stream(const afd_context* c) { return c->stream; }
const afd_mesh_desc& mesh_desc(const afd_mesh* m) { return m->desc; }
int mesh_dof_mask(const afd_mesh* m, uint8_t* host) {
    AFD_HIP_TRY(hipMemcpyAsync(host, m->dofmask, m->g.ndof, hipMemcpyDeviceToHost, m->ctx->stream));
    AFD_HIP_TRY(hipStreamSynchronize(m->ctx->stream));
    return AFD_OK;
}
}  // namespace afd

namespace {

// AFD_COARSE_F32 as read once for the process (-1: not read yet)
int g_coarse_f32 = -1;
// For the FP64 iterations the FP32 copies of the coarse solve matrices are
// opt-in (AFD_COARSE_F32=1 for the process, afd_mesh_coarse_precision per
// mesh): by default they stream the FP64 factor
bool coarse_f32_enabled() {
    if (g_coarse_f32 < 0) {
        const char* e = getenv("AFD_COARSE_F32");
        g_coarse_f32 = (e && *e == '1') ? 1 : 0;
    }
    return g_coarse_f32 == 1;
}
void clear_error() { g_err.clear(); }
bool use_coarse_f32(const afd_mesh* m) { return m->coarse_f32 < 0 ? coarse_f32_enabled() : m->coarse_f32 == 1; }
// The FP32 inner solves of the mixed form stream the FP32 copies unless the
// mesh asks for the FP64 factor: their vectors and products are FP32 already,
// and the FP64 refinement around them sets the accuracy.
bool use_coarse_f32_inner(const afd_mesh* m) { return m->coarse_f32 != 0; }

int check_ctx(afd_context* c) {
    if (!c) {
        set_error("null context");
        return AFD_E_INVALID_ARG;
    }
    AFD_HIP_TRY(hipSetDevice(c->device));
    return AFD_OK;
}

template <typename T>
int dalloc(T** p, size_t n) {
    if (*p) return AFD_OK;
    if (afd::dev_malloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        set_error("device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
        return AFD_E_OOM;
    }
    return AFD_OK;
}
template <typename T>
void dfree(T** p) {
    if (*p) (void)afd::dev_free(*p);
    *p = nullptr;
}

void free_work(Work& w) {
    dfree(&w.X), dfree(&w.R), dfree(&w.P0), dfree(&w.P1), dfree(&w.Q), dfree(&w.Z), dfree(&w.AZ), dfree(&w.F),
        dfree(&w.S), dfree(&w.Ye);
    dfree(&w.Xf), dfree(&w.Rf), dfree(&w.P0f), dfree(&w.P1f), dfree(&w.Qf), dfree(&w.Zf), dfree(&w.AZf),
        dfree(&w.Bf);
    dfree(&w.G), dfree(&w.MU), dfree(&w.sc), dfree(&w.outer), dfree(&w.partM), dfree(&w.partV), dfree(&w.Jdev);
    w.nrhs = 0;
    w.mixed = 0;
}

int ensure_work(afd_mesh* m, int nrhs, int mixed) {
    Work& w = m->w;
    if (w.nrhs >= nrhs && w.mixed >= mixed) return AFD_OK;
    int nr = std::max(nrhs, w.nrhs);
    int mx = std::max(mixed, w.mixed);
    free_work(w);
    const size_t n = (size_t)nr * m->g.ndof;
    AFD_TRY(dalloc(&w.X, n));
    AFD_TRY(dalloc(&w.R, n));
    AFD_TRY(dalloc(&w.P0, n));
    AFD_TRY(dalloc(&w.P1, n));
    AFD_TRY(dalloc(&w.Q, n));
    AFD_TRY(dalloc(&w.Z, n));
    AFD_TRY(dalloc(&w.AZ, n));
    AFD_TRY(dalloc(&w.F, n));
    if (persistent_fits(m->g, m->blk, m->deflate, 1)) AFD_TRY(dalloc(&w.Ye, (size_t)nr * 24 * m->g.nelem));
    if (mx) {
        AFD_TRY(dalloc(&w.Xf, n));
        AFD_TRY(dalloc(&w.Rf, n));
        AFD_TRY(dalloc(&w.P0f, n));
        AFD_TRY(dalloc(&w.P1f, n));
        AFD_TRY(dalloc(&w.Qf, n));
        AFD_TRY(dalloc(&w.Zf, n));
        AFD_TRY(dalloc(&w.AZf, n));
        AFD_TRY(dalloc(&w.Bf, n));
    }
    AFD_TRY(dalloc(&w.G, (size_t)4 * std::max(1, m->blk.ncoarse)));
    AFD_TRY(dalloc(&w.MU, (size_t)4 * std::max(1, m->blk.ncoarse)));
    AFD_TRY(dalloc(&w.sc, 4));
    AFD_TRY(dalloc(&w.outer, 4));
    AFD_TRY(dalloc(&w.partM, (size_t)8 * m->npartM));
    AFD_TRY(dalloc(&w.partV, (size_t)8 * VEC_NPART));
    AFD_TRY(dalloc(&w.Jdev, 4));
    w.nrhs = nr;
    w.mixed = mx;
    return AFD_OK;
}

MatvecArgs mv_args(afd_mesh* m) {
    MatvecArgs a;
    a.g = m->g;
    a.rho = m->rho;
    a.rho32 = m->rho32;
    a.nmask = m->nmask;
    a.rho_t = m->rho_t;
    a.rho32_t = m->rho32_t;
    a.fm_t = m->fm_t;
    for (int f = 0; f < 2; ++f) {
        a.apply_variant[f] = m->tune_variant[f];
        a.apply_zc[f] = m->tune_zc[f];
    }
    return a;
}

int ensure_jacobi(afd_mesh* m) {
    if (m->jacobi_valid) return AFD_OK;
    AFD_TRY(launch_node_rsum(m->g, m->rho, m->rinv, m->rinv32, m->ctx->stream));
    m->jacobi_valid = true;
    return AFD_OK;
}

void setup_blocks(afd_mesh* m) {
    Blocks& b = m->blk;
    const int n[3] = {m->g.nx, m->g.ny, m->g.nz};
    const int bb[3] = {m->desc.bx, m->desc.by, m->desc.bz};
    m->deflate = (bb[0] > 0 && bb[1] > 0 && bb[2] > 0) ? 1 : 0;
    b = Blocks{};
    if (!m->deflate) return;
    int mx = 0;
    for (int a = 0; a < 3; ++a) {
        b.b[a] = std::min(bb[a], n[a]);
        b.nb[a] = (n[a] + b.b[a] - 1) / b.b[a];
        mx = std::max(mx, b.b[a]);
    }
    b.inv_scale = 1.0 / mx;
    b.nblk = b.nb[0] * b.nb[1] * b.nb[2];
    b.ncoarse = 6 * b.nblk;
    int ax[3] = {0, 1, 2};
    std::stable_sort(ax, ax + 3, [&](int p, int q) { return b.nb[p] < b.nb[q]; });
    for (int a = 0; a < 3; ++a) b.perm[a] = ax[a];
    const int n0 = b.nb[ax[0]], n1 = b.nb[ax[1]];
    b.w = 6 * (n0 * n1 + n0 + 1) + 5;
    const int P = choose_coarse_P(b.ncoarse, b.w);
    b.P = P;
    b.K = (b.ncoarse + P - 1) / P;
    b.m = (b.K - 1) / 2;
}

// read at every assembly (once per coarse setup)
bool coarse_probe_forced() {
    const char* e = getenv("AFD_COARSE_ASSEMBLY");
    return e && std::string(e) == "probe";
}

// E = W^T A W into the coarse buffers (not factored).  Default: directly from
// the element matrices of the block-interface elements.  AFD_COARSE_ASSEMBLY=
// probe takes the matrix-free route instead: 27 colors of a 3x3x3 block
// pattern x 6 motions, each an operator apply and a restriction.
int assemble_coarse(afd_mesh* m) {
    hipStream_t s = m->ctx->stream;
    if (!m->coarse.D) {
        m->coarse.blk = m->blk;
        AFD_TRY(coarse_alloc(m->coarse, m->ctx->stream));
    }
    AFD_TRY(coarse_begin(m->coarse, s));
    if (!coarse_probe_forced()) {
        const bool rigid = m->desc.hx == m->desc.hy && m->desc.hy == m->desc.hz;
        return coarse_direct(m->coarse, m->g, m->rho, m->nmask, m->ke_dev, rigid, s);
    }
    AFD_TRY(ensure_work(m, 1, 0));
    MatvecArgs a = mv_args(m);
    for (int color = 0; color < 27; ++color) {
        const int cc[3] = {color % 3, (color / 3) % 3, color / 9};
        if (cc[0] >= m->blk.nb[0] || cc[1] >= m->blk.nb[1] || cc[2] >= m->blk.nb[2]) continue;
        for (int mode = 0; mode < 6; ++mode) {
            AFD_TRY(launch_probe_vector(m->g, m->blk, m->nmask, color, mode, m->w.Z, s));
            AFD_TRY(launch_apply(a, m->kh, 0, 1, m->w.Z, m->w.AZ, s));
            AFD_TRY(launch_restrict(m->g, m->blk, m->nmask, 1, m->w.AZ, m->w.G, s));
            AFD_TRY(coarse_scatter_probe(m->coarse, m->w.G, color, mode, s));
        }
    }
    return AFD_OK;
}

int ensure_coarse(afd_mesh* m) {
    if (!m->deflate) return AFD_OK;
    if (m->coarse.valid) return AFD_OK;
    hipStream_t s = m->ctx->stream;
    AFD_TRY(assemble_coarse(m));
    return coarse_factor(m->coarse, s);
}

int host_or_dev_to_dev(afd_mesh* m, const void* src, size_t bytes, int mem_kind, void* dst) {
    AFD_HIP_TRY(hipMemcpyAsync(dst, src, bytes, mem_kind == AFD_MEM_HOST ? hipMemcpyHostToDevice
                                                                         : hipMemcpyDeviceToDevice,
                               m->ctx->stream));
    if (mem_kind == AFD_MEM_HOST) AFD_HIP_TRY(hipStreamSynchronize(m->ctx->stream));
    return AFD_OK;
}

DcgArgs dcg_args(afd_mesh* m, CgScalars* sc, double* part, int npart) {
    DcgArgs d;
    d.rinv = m->rinv;
    d.sc = sc;
    d.partial = part;
    d.npart = npart;
    return d;
}

// Deflated Jacobi-PCG on A X = B: x0 = W E^-1 W^T b, r0 = b - A x0, then
// q = A p, alpha = r.z/p.q, x += alpha p, r -= alpha q, z = M^-1 r,
// beta = r.z_new/r.z, mu = E^-1 W^T (A z - r), p = beta p + z - W mu
// (Saad et al.'s deflated CG with the coarse correction in A-DEF2 form).
// warm (FP64 only): X holds a start x on entry and the iteration starts from
// x0 = x + W E^-1 W^T (b - A x), the start that keeps W^T r0 = 0 for any x
// (a restart from the current iterate is such a warm start).
// FP64 (T = double) or FP32 vectors (T = float, inner solve of the mixed form);
// dot products and the coarse problem are always FP64.
template <typename T>
int dcg_run(afd_mesh* m, int nrhs, const T* Bv, T* X, T* R, T* P0, T* P1, T* Q, T* Z, T* AZ, CgScalars* sc,
            double rtol, int max_iter, int check_every, const CgScalars* outer_mask, bool warm = false) {
    hipStream_t s = m->ctx->stream;
    Work& w = m->w;
    MatvecArgs a = mv_args(m);
    const bool f32 = sizeof(T) == 4;
    const bool c32 = (f32 ? use_coarse_f32_inner(m) : use_coarse_f32(m)) && m->coarse.valid32;
    const int64_t ndof = m->g.ndof;
    // ||b||
    if constexpr (sizeof(T) == 8) AFD_TRY(launch_dot_rhs(ndof, nrhs, (const double*)Bv, w.partV, VEC_NPART, s));
    else AFD_TRY(launch_dot_rhs_f32(ndof, nrhs, (const float*)Bv, w.partV, VEC_NPART, s));
    AFD_TRY(launch_cg_init(sc, nrhs, w.partV, VEC_NPART, rtol, max_iter, s));
    (void)outer_mask;
    if (warm) {
        // x0 = x + W E^-1 W^T (b - A x), zero on fixed DOFs
        if constexpr (sizeof(T) == 8) {
            AFD_TRY(launch_prolong_add(m->g, m->blk, m->nmask, nrhs, nullptr, sc, X, s));
            if (m->deflate) {
                DcgArgs d0 = dcg_args(m, sc, w.partM, m->npartM);
                AFD_TRY(launch_residual(a, m->kh, d0, nrhs, Bv, X, R, s));
                AFD_TRY(launch_restrict(m->g, m->blk, m->nmask, nrhs, R, w.G, s));
                AFD_TRY(coarse_solve(m->coarse, nrhs, w.G, w.MU, s, c32));
                AFD_TRY(launch_prolong_add(m->g, m->blk, m->nmask, nrhs, w.MU, sc, X, s));
            }
        } else {
            set_error("solve: warm start needs FP64 vectors");
            return AFD_E_INVALID_ARG;
        }
    } else if (m->deflate) {
        // deflated start
        if constexpr (sizeof(T) == 8) AFD_TRY(launch_restrict(m->g, m->blk, m->nmask, nrhs, Bv, w.G, s));
        else AFD_TRY(launch_restrict_f32(m->g, m->blk, m->nmask, nrhs, Bv, w.G, s));
        AFD_TRY(coarse_solve(m->coarse, nrhs, w.G, w.MU, s, c32));
        if constexpr (sizeof(T) == 8) AFD_TRY(launch_prolong(m->g, m->blk, m->nmask, nrhs, w.MU, X, s));
        else AFD_TRY(launch_prolong_f32(m->g, m->blk, m->nmask, nrhs, w.MU, X, s));
    } else {
        if constexpr (sizeof(T) == 8) AFD_TRY(launch_fill_f64(nrhs * ndof, 0.0, (double*)X, s));
        else AFD_TRY(launch_fill_f32(nrhs * ndof, 0.0f, (float*)X, s));
    }
    DcgArgs dm = dcg_args(m, sc, w.partM, m->npartM);
    if constexpr (sizeof(T) == 8) AFD_TRY(launch_residual(a, m->kh, dm, nrhs, Bv, X, R, s));
    else AFD_TRY(launch_residual_f32(a, m->kh, dm, m->rinv32, nrhs, Bv, X, R, s));
    AFD_TRY(launch_cg_start(sc, nrhs, w.partM, m->npartM, s));
    // coarse correction mu = E^-1 W^T (A z - r): the A-DEF2 form of the
    // deflated preconditioner (equal to the Saad form, where W^T r = 0, in
    // exact arithmetic; it removes any rounding drift of W^T r, which the
    // FP32 inner solve of the mixed form needs)
    // The restriction also writes the coarse solve's permuted input (no
    // permutation launch) and, inside the iteration (with_beta), does the CG
    // beta/convergence update that follows the x/r update (no launch of its own).
    auto coarse_of_z = [&](bool with_beta) -> int {
        if (!m->deflate) return AFD_OK;
        const int64_t npad = (int64_t)m->blk.K * m->blk.P;
        CgScalars* bsc = with_beta ? sc : nullptr;
        if constexpr (sizeof(T) == 8) {
            AFD_TRY(launch_apply(a, m->kh, 0, nrhs, Z, AZ, s));
            AFD_TRY(launch_restrict_diff(m->g, m->blk, m->nmask, nrhs, AZ, R, w.G, s, m->coarse.perm,
                                         m->coarse.gperm, npad, bsc, w.partV, VEC_NPART));
        } else {
            AFD_TRY(launch_apply(a, m->kh, 1, nrhs, Z, AZ, s));
            AFD_TRY(launch_restrict_diff_f32(m->g, m->blk, m->nmask, nrhs, AZ, R, w.G, s, m->coarse.perm,
                                             m->coarse.gperm, npad, bsc, w.partV, VEC_NPART));
        }
        return coarse_solve(m->coarse, nrhs, w.G, w.MU, s, c32, true);
    };
    // p' = beta p + M^-1 r - W mu (Pnew), then q = A p' with the p'.q partials;
    // with Xu the same launch applies the iteration's x += alpha p (p = Pold)
    auto direction = [&](T* Pold, T* Pnew, T* Xu) -> int {
        const double* mu = m->deflate ? w.MU : nullptr;
        if constexpr (sizeof(T) == 8)
            AFD_TRY(launch_form_dir(m->g, m->blk, m->nmask, m->kh, sc, nrhs, mu, m->rinv, Pold, R, Pnew, Xu, s));
        else
            AFD_TRY(
                launch_form_dir_f32(m->g, m->blk, m->nmask, m->kh, sc, nrhs, mu, m->rinv32, Pold, R, Pnew, Xu, s));
        return launch_apply_dot(a, m->kh, dm, sizeof(T) == 4 ? 1 : 0, nrhs, Pnew, Q, s);
    };
    if (m->deflate) {
        if constexpr (sizeof(T) == 8) AFD_TRY(launch_precond(m->g, m->kh, m->rinv, nrhs, R, Z, s));
        else AFD_TRY(launch_precond_f32(m->g, m->kh, m->rinv32, nrhs, R, Z, s));
        AFD_TRY(coarse_of_z(false));
    }
    if constexpr (sizeof(T) == 8) AFD_TRY(launch_fill_f64(nrhs * ndof, 0.0, (double*)P0, s));
    else AFD_TRY(launch_fill_f32(nrhs * ndof, 0.0f, (float*)P0, s));
    AFD_TRY(direction(P0, P1, nullptr));
    std::swap(P0, P1);
    std::vector<CgScalars> hsc(nrhs);
    const int ce = std::max(1, check_every);
    auto iterate = [&](int n) -> int {
        for (int j = 0; j < n; ++j) {
            // alpha, r -= alpha q, z, r.z and r.r here; x += alpha p in the direction launch below
            if constexpr (sizeof(T) == 8)
                AFD_TRY(launch_cg_update(m->g, m->kh, m->rinv, sc, nrhs, nullptr, nullptr, R, Q,
                                         m->deflate ? Z : nullptr, w.partV, VEC_NPART, w.partM, m->npartM, s));
            else
                AFD_TRY(launch_cg_update_f32(m->g, m->kh, m->rinv32, sc, nrhs, nullptr, nullptr, R, Q,
                                             m->deflate ? Z : nullptr, w.partV, VEC_NPART, w.partM, m->npartM, s));
            if (!m->deflate || m->blk.nblk < nrhs) AFD_TRY(launch_scalar_beta(sc, nrhs, w.partV, VEC_NPART, s));
            AFD_TRY(coarse_of_z(m->deflate && m->blk.nblk >= nrhs));
            AFD_TRY(direction(P0, P1, X));
            std::swap(P0, P1);
        }
        return AFD_OK;
    };
    // The ce iterations between host convergence checks only launch kernels
    // (iterations past convergence are no-ops on X and R, each kernel checks
    // the per-RHS done flag), so they are recorded once as a HIP graph and
    // replayed; an even ce leaves the direction buffers where they started.
    // The graph is kept on the mesh and re-recorded when any buffer, size or
    // launch configuration baked into it changes.
    const bool graphs = m->ctx->graphs && ce >= 2 && ce % 2 == 0;
    IterGraph& gr = m->graphs[sizeof(T) == 4 ? 1 : 0];
    if (graphs) {
        const Coarse& c = m->coarse;
        const std::vector<uintptr_t> key = {
            (uintptr_t)nrhs, (uintptr_t)ce, (uintptr_t)m->deflate, (uintptr_t)X, (uintptr_t)R, (uintptr_t)P0,
            (uintptr_t)P1, (uintptr_t)Q, (uintptr_t)Z, (uintptr_t)AZ, (uintptr_t)sc, (uintptr_t)w.G,
            (uintptr_t)w.MU, (uintptr_t)w.partM, (uintptr_t)w.partV, (uintptr_t)m->npartM, (uintptr_t)c.Linv,
            (uintptr_t)c.LinvT, (uintptr_t)c.T, (uintptr_t)c.U, (uintptr_t)c.perm, (uintptr_t)c.iperm,
            (uintptr_t)c.gperm, (uintptr_t)c.xperm, (uintptr_t)c.blk.P, (uintptr_t)c.blk.K,
            (uintptr_t)c.Linv32, (uintptr_t)c.LinvT32, (uintptr_t)c.T32, (uintptr_t)c.U32,
            (uintptr_t)c32,
            (uintptr_t)(m->tune_variant[0] + 8), (uintptr_t)(m->tune_variant[1] + 8), (uintptr_t)m->tune_zc[0],
            (uintptr_t)m->tune_zc[1]};
        if (!gr.exec || gr.key != key) {
            // no allocation or free anywhere in the library, and no other
            // recording, while this stream captures (see device_memory_mutex)
            std::lock_guard<std::recursive_mutex> lk(afd::device_memory_mutex());
            gr.release();
            AFD_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            T *p0 = P0, *p1 = P1;
            const int rc = iterate(ce);
            P0 = p0, P1 = p1;
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(s, &graph);
            if (rc != AFD_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            AFD_HIP_TRY(ec);
            const hipError_t ei = hipGraphInstantiate(&gr.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            AFD_HIP_TRY(ei);
            gr.key = key;
        }
    }
    for (int it = 0; it < max_iter; it += ce) {
        const int n = std::min(ce, max_iter - it);
        if (graphs && n == ce) AFD_HIP_TRY(hipGraphLaunch(gr.exec, s));
        else AFD_TRY(iterate(n));
        AFD_HIP_TRY(hipMemcpyAsync(hsc.data(), sc, nrhs * sizeof(CgScalars), hipMemcpyDeviceToHost, s));
        AFD_HIP_TRY(hipStreamSynchronize(s));
        bool all = true;
        for (int r = 0; r < nrhs; ++r) all = all && hsc[r].done != 0;
        if (all) break;
    }
    (void)f32;
    return AFD_OK;
}

}  // namespace

namespace afd {
// afd_modal, optionally starting from (and handing back) the subspace block
// of an earlier run
int modal_with_block(afd_mesh* m, const afd_solve_opts* inner, int nev, double tol, int max_iter, double* lam,
                     double* Phi, double* S, afd_modal_stats* st, EigenBlock* block) {
    if (!m) {
        set_error("modal: null mesh");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    if (st) memset(st, 0, sizeof(*st));
    const double h[3] = {m->desc.hx, m->desc.hy, m->desc.hz};
    return modal_subspace(m, m->g, h, m->rho, m->nmask, inner, nev, tol, max_iter, lam, Phi, S, st, m->ctx->stream,
                          block);
}
// afd_buckling, optionally starting from (and handing back) a subspace block
int buckling_with_block(afd_mesh* m, const double* U, const afd_solve_opts* inner, int nev, double tol, int max_iter,
                        double* lam, double* Phi, double* S, afd_modal_stats* st, EigenBlock* block) {
    if (!m) {
        set_error("buckling: null mesh");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    if (st) memset(st, 0, sizeof(*st));
    const double h[3] = {m->desc.hx, m->desc.hy, m->desc.hz};
    return buckling_subspace(m, m->g, h, m->desc.E, m->desc.nu, m->rho, m->nmask, U, inner, nev, tol, max_iter, lam,
                             Phi, S, st, m->ctx->stream, block);
}
}  // namespace afd

extern "C" {

const char* afd_last_error(void) { return g_err.c_str(); }

int afd_context_create(int device, void* hip_stream, afd_context** out) {
    if (!out) {
        set_error("null output pointer");
        return AFD_E_INVALID_ARG;
    }
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        set_error("no HIP device");
        return AFD_E_NO_DEVICE;
    }
    if (device < 0 || device >= n) {
        set_error("device index out of range");
        return AFD_E_NO_DEVICE;
    }
    AFD_HIP_TRY(hipSetDevice(device));
    afd_context* c = new afd_context();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            set_error("hipStreamCreate failed");
            return AFD_E_HIP;
        }
        c->own_stream = true;
    }
    if (afd::dev_malloc((void**)&c->scratch, VEC_NPART * sizeof(double)) != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        set_error("device allocation failed");
        return AFD_E_OOM;
    }
    // device address of this GPU's static work space of afd_threshold_noalloc
    const int rc = threshold_scratch_init(device);
    if (rc != AFD_OK) {
        (void)afd::dev_free(c->scratch);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return rc;
    }
    *out = c;
    return AFD_OK;
}

void afd_context_destroy(afd_context* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->scratch) (void)afd::dev_free(c->scratch);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int afd_context_use_graphs(afd_context* c, int32_t enable) {
    if (!c) {
        set_error("null context");
        return AFD_E_INVALID_ARG;
    }
    c->graphs = enable != 0;
    return AFD_OK;
}

int afd_context_sync(afd_context* c) {
    AFD_TRY(check_ctx(c));
    AFD_HIP_TRY(hipStreamSynchronize(c->stream));
    return AFD_OK;
}

int afd_mesh_create(afd_context* ctx, const afd_mesh_desc* d, afd_mesh** out) {
    AFD_TRY(check_ctx(ctx));
    if (!d || !out) {
        set_error("null argument");
        return AFD_E_INVALID_ARG;
    }
    *out = nullptr;
    AFD_TRY(validate_desc(*d));
    const int64_t nnode = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
    afd_mesh* m = new afd_mesh();
    m->ctx = ctx;
    m->desc = *d;
    m->g.nx = d->nx;
    m->g.ny = d->ny;
    m->g.nz = d->nz;
    m->g.nnode = nnode;
    m->g.nelem = (int64_t)d->nx * d->ny * d->nz;
    m->g.ndof = 3 * nnode;
    const double h[3] = {d->hx, d->hy, d->hz};
    m->kh = make_ke_haar(h, d->E, d->nu);
    setup_blocks(m);
    m->npartM = matvec_num_tiles(m->g);
    std::vector<double> ke(576);
    make_ke_dense(h, d->E, d->nu, ke.data());
    int64_t ntr = 0;
    const int64_t ntm = tile_layout_sizes(m->g, &ntr);
    int rc = AFD_OK;
    if ((rc = dalloc(&m->rho, m->g.nelem)) || (rc = dalloc(&m->rho32, m->g.nelem)) ||
        (rc = dalloc(&m->nmask, m->g.nnode)) || (rc = dalloc(&m->dofmask, m->g.ndof)) ||
        (rc = dalloc(&m->rinv, m->g.nnode)) || (rc = dalloc(&m->rinv32, m->g.nnode)) ||
        (rc = dalloc(&m->ke_dev, 576)) || (rc = dalloc(&m->rho_t, ntr)) || (rc = dalloc(&m->rho32_t, ntr)) ||
        (rc = dalloc(&m->fm_t, ntm))) {
        afd_mesh_destroy(m);
        return rc;
    }
    hipStream_t s = ctx->stream;
    if (launch_fill_f64(m->g.nelem, 1.0, m->rho, s) || launch_fill_f32(m->g.nelem, 1.0f, m->rho32, s) ||
        hipMemsetAsync(m->nmask, 0, m->g.nnode, s) != hipSuccess ||
        launch_tile_rho(m->g, m->rho, m->rho_t, m->rho32_t, s) || launch_tile_fmask(m->g, m->nmask, m->fm_t, s) ||
        hipMemcpyAsync(m->ke_dev, ke.data(), 576 * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        afd_mesh_destroy(m);
        set_error("mesh initialisation failed");
        return AFD_E_HIP;
    }
    *out = m;
    return AFD_OK;
}

void afd_mesh_destroy(afd_mesh* m) {
    if (!m) return;
    (void)hipSetDevice(m->ctx->device);
    (void)hipStreamSynchronize(m->ctx->stream);
    m->graphs[0].release();
    m->graphs[1].release();
    free_work(m->w);
    coarse_free(m->coarse);
    dfree(&m->rho), dfree(&m->rho32), dfree(&m->nmask), dfree(&m->dofmask), dfree(&m->rinv), dfree(&m->rinv32),
        dfree(&m->ke_dev), dfree(&m->rho_t), dfree(&m->rho32_t), dfree(&m->fm_t);
    delete m;
}

int afd_mesh_sizes(const afd_mesh* m, int64_t* ne, int64_t* nn, int64_t* nd, int64_t* nc) {
    if (!m) {
        set_error("null mesh");
        return AFD_E_INVALID_ARG;
    }
    if (ne) *ne = m->g.nelem;
    if (nn) *nn = m->g.nnode;
    if (nd) *nd = m->g.ndof;
    if (nc) *nc = m->deflate ? m->blk.ncoarse : 0;
    return AFD_OK;
}

__global__ void k_rho32(int64_t n, const double* a, float* b) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

int afd_mesh_set_scale(afd_mesh* m, const double* rho, int64_t n, int mem_kind) {
    if (!m || !rho) {
        set_error("null argument");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    if (n != m->g.nelem || (mem_kind != AFD_MEM_HOST && mem_kind != AFD_MEM_DEVICE)) {
        set_error("set_scale: n_elem mismatch or bad mem_kind");
        return AFD_E_INVALID_ARG;
    }
    if (mem_kind == AFD_MEM_HOST)
        for (int64_t i = 0; i < n; ++i)
            if (!(rho[i] > 0.0) || !std::isfinite(rho[i])) {
                set_error("set_scale: rho must be positive and finite (element " + std::to_string(i) + ")");
                return AFD_E_INVALID_ARG;
            }
    AFD_TRY(host_or_dev_to_dev(m, rho, n * sizeof(double), mem_kind, m->rho));
    hipLaunchKernelGGL(k_rho32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->ctx->stream, n, m->rho, m->rho32);
    AFD_HIP_TRY(hipGetLastError());
    AFD_TRY(launch_tile_rho(m->g, m->rho, m->rho_t, m->rho32_t, m->ctx->stream));
    m->jacobi_valid = false;
    m->coarse.valid = false;
    return AFD_OK;
}

int afd_mesh_set_fixed(afd_mesh* m, const uint8_t* mask, int64_t n, int mem_kind) {
    if (!m || !mask) {
        set_error("null argument");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    if (n != m->g.ndof || (mem_kind != AFD_MEM_HOST && mem_kind != AFD_MEM_DEVICE)) {
        set_error("set_fixed: n_dof mismatch or bad mem_kind");
        return AFD_E_INVALID_ARG;
    }
    if (mem_kind == AFD_MEM_HOST) {
        bool any = false;
        for (int64_t i = 0; i < n && !any; ++i) any = mask[i] != 0;
        m->any_fixed = any;
    } else {
        m->any_fixed = true;
    }
    AFD_TRY(host_or_dev_to_dev(m, mask, n, mem_kind, m->dofmask));
    AFD_TRY(launch_pack_mask(m->g, m->dofmask, m->nmask, m->ctx->stream));
    AFD_TRY(launch_tile_fmask(m->g, m->nmask, m->fm_t, m->ctx->stream));
    m->coarse.valid = false;
    return AFD_OK;
}

int afd_mesh_footprint(const afd_mesh* m, int32_t nrhs, int32_t precision, uint64_t* bytes) {
    if (!m || !bytes || nrhs < 1 || nrhs > 4) {
        set_error("footprint: bad argument");
        return AFD_E_INVALID_ARG;
    }
    const uint64_t nd = m->g.ndof, nn = m->g.nnode, ne = m->g.nelem;
    uint64_t b = ne * 12 + nn * (1 + 12) + nd + 576 * 8;                 // rho, rho32, masks, rinv
    int64_t ntr = 0;
    const int64_t ntm = tile_layout_sizes(m->g, &ntr);
    b += (uint64_t)ntr * 12 + (uint64_t)ntm * 2;                         // tile-major apply inputs
    b += (uint64_t)nrhs * nd * 8 * 8;                                    // FP64 work vectors
    if (persistent_fits(m->g, m->blk, m->deflate, 1)) b += (uint64_t)nrhs * ne * 24 * 8;  // persistent form
    if (precision == AFD_MIXED) b += (uint64_t)nrhs * nd * 4 * 8;        // FP32 inner vectors
    if (m->deflate) {
        const uint64_t PP = (uint64_t)m->blk.P * m->blk.P;
        b += PP * m->blk.K * 8 * 6 + PP * 8 * 2 + (uint64_t)m->blk.K * m->blk.P * 8 * 14;  // 2 work blocks
        b += PP * m->blk.K * 4 * 4;                                     // FP32 copies of the solve matrices
    }
    b += (uint64_t)m->npartM * 64 + VEC_NPART * 64;
    *bytes = b;
    return AFD_OK;
}

int afd_mesh_ke(const afd_mesh* m, double* ke) {
    if (!m || !ke) {
        set_error("null argument");
        return AFD_E_INVALID_ARG;
    }
    const double h[3] = {m->desc.hx, m->desc.hy, m->desc.hz};
    make_ke_dense(h, m->desc.E, m->desc.nu, ke);
    return AFD_OK;
}

int afd_mesh_autotune(afd_mesh* m, int32_t precision, int32_t nrhs, afd_tune_report* rep) {
    if (!m || nrhs < 1 || nrhs > 4 || (precision != AFD_FP64 && precision != AFD_FP32)) {
        set_error("autotune: bad argument (nrhs 1..4, precision FP64 or FP32)");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    hipStream_t s = m->ctx->stream;
    const int f = precision == AFD_FP32 ? 1 : 0;
    const size_t word = f ? 4 : 8, n = (size_t)nrhs * m->g.ndof;
    void *U = nullptr, *Y = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (afd::dev_malloc(&U, n * word) != hipSuccess || afd::dev_malloc(&Y, n * word) != hipSuccess) {
        if (U) (void)afd::dev_free(U);
        set_error("autotune: scratch allocation failed");
        return AFD_E_OOM;
    }
    int rc = AFD_OK;
    if (f) rc = launch_fill_f32((int64_t)n, 1.0f, (float*)U, s);
    else rc = launch_fill_f64((int64_t)n, 1.0, (double*)U, s);
    if (rc == AFD_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        set_error("autotune: event creation failed");
        rc = AFD_E_HIP;
    }
    // candidates: each kernel variant at its one-round chunking, and at 1/2,
    // 2, 3 and 4 times as many chunks (more, shorter z chunks trade z overlap
    // for parallelism)
    struct Cand {
        int v, zc;
    };
    std::vector<Cand> cands;
    for (int v : {6, 4, 2, 3, 0}) {
        int zc = 0, nch = 0;
        apply_tiling(m->g, f, v, 0, nrhs, &zc, &nch);
        for (int mult : {2, 1, 4, 6, 8}) {  // chunks x mult / 2
            const int want = std::max(1, nch * mult / 2);
            const int planes = m->g.nz + 1;
            const int z = std::max(1, (planes + want - 1) / want);
            bool dup = false;
            for (const Cand& c : cands) dup = dup || (c.v == v && c.zc == z);
            if (!dup) cands.push_back({v, z});
        }
    }
    auto time_of = [&](int v, int zc, double* us) -> int {
        MatvecArgs a = mv_args(m);
        a.apply_variant[f] = v;
        a.apply_zc[f] = zc;
        for (int i = 0; i < 3; ++i) AFD_TRY(launch_apply(a, m->kh, f, nrhs, U, Y, s));
        const int reps = 10;
        AFD_HIP_TRY(hipEventRecord(e0, s));
        for (int i = 0; i < reps; ++i) AFD_TRY(launch_apply(a, m->kh, f, nrhs, U, Y, s));
        AFD_HIP_TRY(hipEventRecord(e1, s));
        AFD_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        AFD_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        *us = 1e3 * ms / reps;
        return AFD_OK;
    };
    double best_us = 1e30, def_us = 0.0;
    int best_v = -1, best_zc = 0;
    // the apply speeds up over the first few hundred launches of a process
    // (clocks ramping under load): warm up with the default before timing
    if (rc == AFD_OK) {
        MatvecArgs a = mv_args(m);
        a.apply_variant[f] = -1;
        a.apply_zc[f] = 0;
        for (int i = 0; rc == AFD_OK && i < 300; ++i) rc = launch_apply(a, m->kh, f, nrhs, U, Y, s);
    }
    if (rc == AFD_OK) rc = time_of(-1, 0, &def_us);
    for (size_t i = 0; rc == AFD_OK && i < cands.size(); ++i) {
        double us = 0.0;
        rc = time_of(cands[i].v, cands[i].zc, &us);
        if (rc == AFD_OK && us < best_us) {
            best_us = us;
            best_v = cands[i].v;
            best_zc = cands[i].zc;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)afd::dev_free(U);
    (void)afd::dev_free(Y);
    if (rc != AFD_OK) return rc;
    // keep the default unless a candidate is clearly faster (timing noise is
    // a few percent between runs)
    if (!(best_us < 0.97 * def_us)) {
        best_v = -1;
        best_zc = 0;
        best_us = def_us;
    }
    m->tune_variant[f] = best_v;
    m->tune_zc[f] = best_zc;
    if (rep) {
        rep->variant = best_v;
        rep->zc = best_zc;
        rep->us = best_us;
        rep->default_us = def_us;
        rep->ncandidates = (int32_t)cands.size();
    }
    return AFD_OK;
}

int afd_mesh_apply_config(afd_mesh* m, int32_t precision, int32_t variant, int32_t zc) {
    if (!m || (precision != AFD_FP64 && precision != AFD_FP32) ||
        !(variant == -1 || variant == 0 || variant == 2 || variant == 3 || variant == 4 || variant == 6) || zc < 0) {
        set_error("apply_config: bad argument (variant -1, 0, 2, 3, 4 or 6; zc >= 0)");
        return AFD_E_INVALID_ARG;
    }
    const int f = precision == AFD_FP32 ? 1 : 0;
    m->tune_variant[f] = variant;
    m->tune_zc[f] = zc;
    return AFD_OK;
}

int afd_mesh_solver_form(afd_mesh* m, int32_t form) {
    if (!m || (form != AFD_FORM_LAUNCHES && form != AFD_FORM_PERSISTENT)) {
        set_error("solver_form: AFD_FORM_LAUNCHES or AFD_FORM_PERSISTENT");
        return AFD_E_INVALID_ARG;
    }
    m->solver_form = form;
    return AFD_OK;
}

int afd_mesh_coarse_precision(afd_mesh* m, int32_t precision) {
    if (!m || (precision != AFD_FP64 && precision != AFD_FP32)) {
        set_error("coarse_precision: AFD_FP64 or AFD_FP32");
        return AFD_E_INVALID_ARG;
    }
    m->coarse_f32 = precision == AFD_FP32 ? 1 : 0;
    return AFD_OK;
}

int afd_apply_K(afd_mesh* m, int32_t precision, int32_t nrhs, const void* U, void* Y) {
    if (!m || !U || !Y || nrhs < 1 || nrhs > 4 || (precision != AFD_FP64 && precision != AFD_FP32)) {
        set_error("apply_K: bad argument (nrhs 1..4, precision FP64 or FP32)");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    return launch_apply(mv_args(m), m->kh, precision == AFD_FP32, nrhs, U, Y, m->ctx->stream);
}

int afd_apply_K_mfma(afd_mesh* m, int32_t nrhs, const double* U, double* Y) {
    if (!m || !U || !Y || nrhs < 1 || nrhs > 4) {
        set_error("apply_K_mfma: bad argument");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    return launch_apply_mfma(mv_args(m), m->ke_dev, nrhs, U, Y, m->ctx->stream);
}

int afd_jacobi(afd_mesh* m, double* d) {
    if (!m || !d) {
        set_error("null argument");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    AFD_TRY(ensure_jacobi(m));
    return launch_jacobi_full(m->g, m->rinv, m->nmask, m->kh, d, m->ctx->stream);
}

int afd_dot(afd_context* c, int64_t n, const double* x, const double* y, double* out) {
    AFD_TRY(check_ctx(c));
    if (n < 0 || !x || !y || !out) {
        set_error("dot: bad argument");
        return AFD_E_INVALID_ARG;
    }
    return launch_dot(n, x, y, c->scratch, VEC_NPART, out, c->stream);
}

static int need_deflate(afd_mesh* m) {
    if (!m) {
        set_error("null mesh");
        return AFD_E_INVALID_ARG;
    }
    if (!m->deflate) {
        set_error("deflation disabled for this mesh (block size 0)");
        return AFD_E_INVALID_ARG;
    }
    return check_ctx(m->ctx);
}

int afd_restrict(afd_mesh* m, int32_t nrhs, const double* V, double* G) {
    AFD_TRY(need_deflate(m));
    if (nrhs < 1 || nrhs > 4 || !V || !G) {
        set_error("restrict: bad argument");
        return AFD_E_INVALID_ARG;
    }
    return launch_restrict(m->g, m->blk, m->nmask, nrhs, V, G, m->ctx->stream);
}

int afd_prolong(afd_mesh* m, int32_t nrhs, const double* MU, double* V) {
    AFD_TRY(need_deflate(m));
    if (nrhs < 1 || nrhs > 4 || !V || !MU) {
        set_error("prolong: bad argument");
        return AFD_E_INVALID_ARG;
    }
    return launch_prolong(m->g, m->blk, m->nmask, nrhs, MU, V, m->ctx->stream);
}

int afd_coarse_setup(afd_mesh* m, int32_t* dropped) {
    AFD_TRY(need_deflate(m));
    AFD_TRY(ensure_coarse(m));
    if (dropped) *dropped = m->coarse.dropped;
    return AFD_OK;
}

int afd_coarse_matrix(afd_mesh* m, double* E) {
    AFD_TRY(need_deflate(m));
    if (!E || m->blk.ncoarse > 8192) {
        set_error("coarse_matrix: null output or n_coarse > 8192");
        return AFD_E_INVALID_ARG;
    }
    // assemble (without factoring) into the coarse buffers, copy out, invalidate
    hipStream_t s = m->ctx->stream;
    AFD_TRY(assemble_coarse(m));
    int rc = coarse_to_dense_host(m->coarse, E, s);
    m->coarse.valid = false;
    return rc;
}

int afd_coarse_solve(afd_mesh* m, int32_t nrhs, const double* G, double* MU) {
    AFD_TRY(need_deflate(m));
    if (nrhs < 1 || nrhs > 4 || !G || !MU) {
        set_error("coarse_solve: bad argument");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(ensure_coarse(m));
    return coarse_solve(m->coarse, nrhs, G, MU, m->ctx->stream);
}

int afd_sensitivity(afd_mesh* m, int32_t nrhs, const double* U, int32_t npairs, const int32_t* pairs, double* S) {
    if (!m || !U || !S || nrhs < 1 || nrhs > 4 || npairs < 0 || nrhs + npairs > 16 || (npairs > 0 && !pairs)) {
        set_error("sensitivity: bad argument");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    const double* ua[16];
    const double* ub[16];
    for (int f = 0; f < nrhs; ++f) ua[f] = ub[f] = U + (int64_t)f * m->g.ndof;
    for (int p = 0; p < npairs; ++p) {
        const int a = pairs[2 * p], b = pairs[2 * p + 1];
        if (a < 0 || a >= nrhs || b < 0 || b >= nrhs) {
            set_error("sensitivity: pair index out of range");
            return AFD_E_INVALID_ARG;
        }
        ua[nrhs + p] = U + (int64_t)a * m->g.ndof;
        ub[nrhs + p] = U + (int64_t)b * m->g.ndof;
    }
    return launch_sensitivity(m->g, m->kh, m->rho, nrhs + npairs, ua, ub, S, m->ctx->stream);
}

int afd_threshold(afd_context* c, const double* s, const int32_t* tie, int64_t n, double vol_frac, uint8_t* solid,
                  int32_t* order, double* tau) {
    AFD_TRY(check_ctx(c));
    if (!s || !solid) {
        set_error("threshold: null argument");
        return AFD_E_INVALID_ARG;
    }
    return threshold_gpu(s, tie, n, vol_frac, solid, order, tau, c->stream);
}

int afd_threshold_noalloc(afd_context* c, const double* s, const int32_t* tie, int64_t n, double vol_frac,
                          uint8_t* solid, int32_t* order, double* tau) {
    AFD_TRY(check_ctx(c));
    if (!s || !solid) {
        set_error("threshold_noalloc: null argument");
        return AFD_E_INVALID_ARG;
    }
    return threshold_noalloc(c->device, s, tie, n, vol_frac, solid, order, tau, c->stream);
}

int afd_apply_M(afd_mesh* m, int32_t nrhs, const double* U, double* Y) {
    if (!m || !U || !Y) {
        set_error("apply_M: null argument");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    const double h[3] = {m->desc.hx, m->desc.hy, m->desc.hz};
    return mass_apply(m->g, h, m->rho, m->nmask, nrhs, U, Y, m->ctx->stream);
}

int afd_modal(afd_mesh* m, const afd_solve_opts* inner, int32_t nev, double tol, int32_t max_iter, double* lam,
              double* Phi, double* S, afd_modal_stats* st) {
    return afd::modal_with_block(m, inner, nev, tol, max_iter, lam, Phi, S, st, nullptr);
}

int afd_apply_Kg(afd_mesh* m, const double* U0, int32_t nrhs, const double* X, double* Y) {
    if (!m) {
        set_error("apply_Kg: null mesh");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    const double h[3] = {m->desc.hx, m->desc.hy, m->desc.hz};
    return geo_apply(m->g, h, m->desc.E, m->desc.nu, m->rho, m->nmask, U0, nrhs, X, Y, m->ctx->stream);
}

int afd_buckling(afd_mesh* m, const double* U, const afd_solve_opts* inner, int32_t nev, double tol,
                 int32_t max_iter, double* lam, double* Phi, double* S, afd_modal_stats* st) {
    return afd::buckling_with_block(m, U, inner, nev, tol, max_iter, lam, Phi, S, st, nullptr);
}

int afd_stress_pnorm(afd_mesh* m, int32_t nrhs, const double* U, double p, double* vm, double* pn, double* B) {
    if (!m || !U || !pn) {
        set_error("stress_pnorm: null argument");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    const double h[3] = {m->desc.hx, m->desc.hy, m->desc.hz};
    return stress_pnorm(m->g, h, m->desc.E, m->desc.nu, m->rho, m->nmask, nrhs, U, p, vm, pn, B, m->ctx->stream);
}

int afd_combine_fields(afd_context* c, int64_t n, int32_t nterms, const double* const* fields, const int32_t* rows,
                       const double* coef, double* out) {
    AFD_TRY(check_ctx(c));
    if (!fields || !rows || !coef || !out) {
        set_error("combine_fields: null argument");
        return AFD_E_INVALID_ARG;
    }
    return launch_combine(n, nterms, fields, rows, coef, out, c->stream);
}

int afd_casting(afd_context* c, const int32_t dims[3], const double* phi, int32_t axis, int32_t parting,
                double* out, int32_t* dist) {
    AFD_TRY(check_ctx(c));
    if (!dims || !phi || !out || axis < 0 || axis > 2) {
        set_error("casting: null argument or axis outside 0..2");
        return AFD_E_INVALID_ARG;
    }
    const int d[3] = {dims[0], dims[1], dims[2]};
    if (d[0] < 1 || d[1] < 1 || d[2] < 1 || (int64_t)d[0] * d[1] * d[2] >= (int64_t(1) << 31) || parting < 0 ||
        parting > d[axis]) {
        set_error("casting: dims must be >= 1 (fewer than 2^31 elements), parting in 0..dims[axis]");
        return AFD_E_INVALID_ARG;
    }
    if (dist) AFD_TRY(launch_parting_distance(d, axis, parting, dist, c->stream));
    return launch_cast(d, axis, parting, phi, out, c->stream);
}

int afd_solve(afd_mesh* m, const afd_solve_opts* o, int32_t nrhs, const double* F, double* U, double* J, double* S,
              afd_solve_stats* st) {
    if (!m || !o || !F || !U || nrhs < 1 || nrhs > 4) {
        set_error("solve: bad argument (nrhs 1..4, non-null F, U, opts)");
        return AFD_E_INVALID_ARG;
    }
    AFD_TRY(check_ctx(m->ctx));
    if (!(o->rtol > 0) || o->max_iter < 1 || (o->precision != AFD_FP64 && o->precision != AFD_MIXED) ||
        (o->mem_kind != AFD_MEM_HOST && o->mem_kind != AFD_MEM_DEVICE) || o->npairs < 0 ||
        nrhs + o->npairs > 16 || (o->npairs > 0 && !o->pairs)) {
        set_error("solve: bad options");
        return AFD_E_INVALID_ARG;
    }
    for (int p = 0; p < o->npairs; ++p)
        if (o->pairs[2 * p] < 0 || o->pairs[2 * p] >= nrhs || o->pairs[2 * p + 1] < 0 ||
            o->pairs[2 * p + 1] >= nrhs) {
            set_error("solve: pair index out of range");
            return AFD_E_INVALID_ARG;
        }
    const int64_t ndof = m->g.ndof;
    const bool host = o->mem_kind == AFD_MEM_HOST;
    if (host) {
        std::vector<uint8_t> mask(ndof);
        AFD_HIP_TRY(hipMemcpyAsync(mask.data(), m->dofmask, ndof, hipMemcpyDeviceToHost, m->ctx->stream));
        AFD_HIP_TRY(hipStreamSynchronize(m->ctx->stream));
        for (int r = 0; r < nrhs; ++r)
            for (int64_t i = 0; i < ndof; ++i) {
                const double f = F[r * ndof + i];
                if (!std::isfinite(f) || (m->any_fixed && mask[i] && f != 0.0)) {
                    set_error("solve: F must be finite and zero on fixed DOFs");
                    return AFD_E_INVALID_ARG;
                }
            }
    }
    hipStream_t s = m->ctx->stream;
    const bool mixed = o->precision == AFD_MIXED;
    const double t0 = now_s();
    AFD_TRY(ensure_work(m, nrhs, mixed ? 1 : 0));
    AFD_TRY(ensure_jacobi(m));
    AFD_TRY(ensure_coarse(m));
    Work& w = m->w;
    AFD_HIP_TRY(hipMemcpyAsync(w.F, F, nrhs * ndof * sizeof(double),
                               host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    AFD_HIP_TRY(hipStreamSynchronize(s));
    const double t1 = now_s();
    const int ce = o->check_every > 0 ? o->check_every : 16;
    std::vector<CgScalars> hsc(nrhs), hout(nrhs);
    int refinements = 0;
    // FP32 copies of the coarse solve matrices for the iterations that stream
    // them (made once per factorisation; without memory for them the FP64
    // factor is used)
    if (m->deflate && (use_coarse_f32(m) || (mixed && use_coarse_f32_inner(m))) && coarse_make_f32(m->coarse, s) != AFD_OK)
        clear_error();
    // warm start: the caller's x0 (host or device per mem_kind; its values on
    // fixed DOFs are ignored)
    const bool warm = o->x0 != nullptr;
    if (warm)
        AFD_HIP_TRY(hipMemcpyAsync(w.X, o->x0, nrhs * ndof * sizeof(double),
                                   host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    // true FP64 residual r = f - A x: rr[r] = ||r||^2, bb[r] = ||f||^2 (host sums of
    // the kernels' fixed-order partials)
    std::vector<double> rr(nrhs), bb(nrhs);
    auto true_residual = [&]() -> int {
        AFD_TRY(launch_dot_rhs(ndof, nrhs, w.F, w.partV, VEC_NPART, s));
        std::vector<double> part(2 * nrhs * VEC_NPART);
        AFD_HIP_TRY(hipMemcpyAsync(part.data(), w.partV, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        // residual with a scalar set that is not done
        std::vector<CgScalars> zero(nrhs);
        memset(zero.data(), 0, nrhs * sizeof(CgScalars));
        AFD_HIP_TRY(hipMemcpyAsync(w.outer, zero.data(), nrhs * sizeof(CgScalars), hipMemcpyHostToDevice, s));
        DcgArgs dm = dcg_args(m, w.outer, w.partM, m->npartM);
        AFD_TRY(launch_residual(mv_args(m), m->kh, dm, nrhs, w.F, w.X, w.Z, s));
        std::vector<double> pm(2 * nrhs * (size_t)m->npartM);
        AFD_HIP_TRY(hipMemcpyAsync(pm.data(), w.partM, pm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        AFD_HIP_TRY(hipStreamSynchronize(s));
        for (int r = 0; r < nrhs; ++r) {
            double b = 0, q = 0;
            for (int i = 0; i < VEC_NPART; ++i) b += part[(size_t)(r * 2 + 1) * VEC_NPART + i];
            for (int i = 0; i < m->npartM; ++i) q += pm[(size_t)(r * 2 + 1) * m->npartM + i];
            bb[r] = b;
            rr[r] = q;
        }
        return AFD_OK;
    };
    auto truly_converged = [&](int r) { return bb[r] == 0.0 || rr[r] <= o->rtol * o->rtol * bb[r]; };
    if (!mixed) {
        // The iteration stops on its recursive residual at 0.99 rtol (it drifts
        // from the true residual by ~1e-5 relative on these meshes; the margin
        // costs < 1 iteration).  The true FP64 residual then decides: a column
        // above rtol is restarted from its current iterate (a warm start, so
        // the recursive residual restarts from the true one), at most
        // FP64_RESTARTS times within the max_iter budget; a column still above
        // rtol after that has met the FP64 attainable accuracy of its problem
        // and is reported AFD_E_NOT_CONVERGED.
        constexpr int FP64_RESTARTS = 3;
        // the execution form (the iteration is the same): the graph-recorded
        // launch chain, or one launch per solve on request
        const bool persistent = m->solver_form == AFD_FORM_PERSISTENT;
        if (persistent && !(persistent_fits(m->g, m->blk, m->deflate, nrhs) && w.Ye)) {
            set_error("solve: the persistent form needs at most " + std::to_string(PERSISTENT_MAX_ELEMS) +
                      " elements and a coarse problem of one super-block");
            return AFD_E_INVALID_ARG;
        }
        const Coarse& cf = m->coarse;
        std::vector<int> iters(nrhs, 0);
        for (int run = 0;; ++run) {
            int used = 0;
            for (int r = 0; r < nrhs; ++r) used = std::max(used, iters[r]);
            if (persistent)
                AFD_TRY(launch_dcg_persistent(m->g, m->blk, m->deflate, m->kh, m->rho, m->nmask, m->rinv, cf.Linv,
                                              cf.LinvT, cf.perm, cf.iperm, nrhs, w.F, w.X, w.R, w.P0, w.Q, w.Z, w.Ye,
                                              w.sc, 0.99 * o->rtol, std::max(1, o->max_iter - used), warm || run > 0,
                                              s));
            else
                AFD_TRY(dcg_run<double>(m, nrhs, w.F, w.X, w.R, w.P0, w.P1, w.Q, w.Z, w.AZ, w.sc, 0.99 * o->rtol,
                                        std::max(1, o->max_iter - used), ce, nullptr, warm || run > 0));
            AFD_HIP_TRY(hipMemcpyAsync(hsc.data(), w.sc, nrhs * sizeof(CgScalars), hipMemcpyDeviceToHost, s));
            AFD_TRY(true_residual());  // synchronises
            bool again = false;
            for (int r = 0; r < nrhs; ++r) {
                iters[r] += hsc[r].iters;
                if (hsc[r].done == 1 && !truly_converged(r)) again = true;
            }
            used = 0;
            for (int r = 0; r < nrhs; ++r) used = std::max(used, iters[r]);
            if (!again || run >= FP64_RESTARTS || used >= o->max_iter) break;
            refinements = run + 1;
            if (verbose())
                for (int r = 0; r < nrhs; ++r)
                    fprintf(stderr, "[afd] restart %d rhs %d: true |r|/|f| %.3e after %d it\n", run + 1, r,
                            std::sqrt(rr[r] / std::max(bb[r], 1e-300)), iters[r]);
        }
        for (int r = 0; r < nrhs; ++r) hsc[r].iters = iters[r];
    } else {
        // FP64 iterative refinement around an FP32 deflated PCG
        MatvecArgs a = mv_args(m);
        const int max_ref = o->max_refine > 0 ? o->max_refine : 30;
        const double inner = (o->inner_rtol > 0 && o->inner_rtol < 1) ? o->inner_rtol : 1e-4;
        AFD_TRY(launch_dot_rhs(ndof, nrhs, w.F, w.partV, VEC_NPART, s));
        AFD_TRY(launch_cg_init(w.outer, nrhs, w.partV, VEC_NPART, o->rtol, max_ref, s));
        if (warm) AFD_TRY(launch_prolong_add(m->g, m->blk, m->nmask, nrhs, nullptr, w.outer, w.X, s));
        else AFD_TRY(launch_fill_f64(nrhs * ndof, 0.0, w.X, s));
        int total_inner = 0;
        std::vector<int> inner_iters(nrhs, 0), stall(nrhs, 0);
        std::vector<double> prev_rr(nrhs, 0.0);
        for (int ref = 0; ref <= max_ref; ++ref) {
            DcgArgs dm = dcg_args(m, w.outer, w.partM, m->npartM);
            // residual r = f - A x in FP64 (partials: slot 1 = r.r); the outer
            // scalars are not "done" yet for RESID unless converged
            AFD_TRY(launch_residual(a, m->kh, dm, nrhs, w.F, w.X, w.R, s));
            AFD_TRY(launch_outer_norm(w.outer, nrhs, w.partM, m->npartM, s));
            AFD_HIP_TRY(hipMemcpyAsync(hout.data(), w.outer, nrhs * sizeof(CgScalars), hipMemcpyDeviceToHost, s));
            AFD_HIP_TRY(hipStreamSynchronize(s));
            bool all = true;
            for (int r = 0; r < nrhs; ++r) all = all && hout[r].done != 0;
            if (all) break;
            refinements = ref + 1;
            AFD_TRY(launch_to_f32_scaled(ndof, nrhs, w.R, w.outer, w.Bf, s));
            // the FP32 inner solve reduces the residual by inner_rtol in the first
            // sweep; later sweeps by what is still missing to the outer target
            // (with a factor 2 of margin), within [max(inner_rtol / 100, 1e-6),
            // 1/2] (FP32 inner solves here reach 3e-6 reliably), so that the
            // refinement usually needs two sweeps and the last one does not solve
            // far past rtol.  Past a few hundred iterations FP32 CG has
            // stagnated, so cap it.
            double inner_k = inner;
            if (ref > 0) {
                double rel_max = 0.0;
                for (int r = 0; r < nrhs; ++r)
                    if (hout[r].done == 0 && hout[r].bb > 0)
                        rel_max = std::max(rel_max, std::sqrt(hout[r].rr / hout[r].bb));
                const double floor_k = std::max(0.01 * inner, 1e-6);
                if (rel_max > 0) inner_k = std::min(0.5, std::max(floor_k, 0.5 * o->rtol / rel_max));
            }
            const int inner_max = std::min(o->max_iter, 1000);
            AFD_TRY(dcg_run<float>(m, nrhs, w.Bf, w.Xf, w.Rf, w.P0f, w.P1f, w.Qf, w.Zf, w.AZf, w.sc, inner_k,
                                   inner_max, ce, w.outer));
            AFD_HIP_TRY(hipMemcpyAsync(hsc.data(), w.sc, nrhs * sizeof(CgScalars), hipMemcpyDeviceToHost, s));
            AFD_HIP_TRY(hipStreamSynchronize(s));
            for (int r = 0; r < nrhs; ++r) {
                inner_iters[r] += hsc[r].iters;
                total_inner += hsc[r].iters;
                if (verbose())
                    fprintf(stderr, "[afd] sweep %d rhs %d: outer |r|/|f| %.3e, inner %d it, inner status %d\n", ref,
                            r, std::sqrt(hout[r].rr / std::max(hout[r].bb, 1e-300)), hsc[r].iters, hsc[r].done);
                // stagnation of the outer residual: stop this column
                if (hout[r].done == 0) {
                    if (prev_rr[r] > 0 && hout[r].rr > 0.81 * prev_rr[r]) ++stall[r];
                    else stall[r] = 0;
                    prev_rr[r] = hout[r].rr;
                    if (stall[r] >= 3) {
                        hout[r].done = 3;
                        AFD_HIP_TRY(hipMemcpyAsync(&w.outer[r].done, &hout[r].done, sizeof(int32_t),
                                                   hipMemcpyHostToDevice, s));
                    }
                }
            }
            AFD_TRY(launch_axpy_refine(ndof, nrhs, w.outer, w.Xf, w.X, s));
        }
        for (int r = 0; r < nrhs; ++r) {
            hsc[r] = hout[r];
            hsc[r].iters = inner_iters[r];
        }
        (void)total_inner;
        AFD_TRY(true_residual());
    }
    AFD_HIP_TRY(hipStreamSynchronize(s));
    const double t2 = now_s();
    // compliance, energies (the true FP64 residual of the returned X is in rr, bb)
    std::vector<double> Jh(nrhs);
    {
        for (int r = 0; r < nrhs; ++r) AFD_TRY(launch_dot(ndof, w.F + r * ndof, w.X + r * ndof, m->ctx->scratch,
                                                           VEC_NPART, w.Jdev + r, s));
        AFD_HIP_TRY(hipMemcpyAsync(Jh.data(), w.Jdev, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        AFD_HIP_TRY(hipStreamSynchronize(s));
    }
    if (host) {
        AFD_HIP_TRY(hipMemcpyAsync(U, w.X, nrhs * ndof * sizeof(double), hipMemcpyDeviceToHost, s));
        if (J) memcpy(J, Jh.data(), nrhs * sizeof(double));
    } else {
        AFD_HIP_TRY(hipMemcpyAsync(U, w.X, nrhs * ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (J) AFD_HIP_TRY(hipMemcpyAsync(J, w.Jdev, nrhs * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    if (S) {
        const int nf = nrhs + o->npairs;
        double* Sd = S;
        if (host) {
            dfree(&w.S);
            AFD_TRY(dalloc(&w.S, (size_t)nf * m->g.nelem));
            Sd = w.S;
        }
        const double* ua[16];
        const double* ub[16];
        for (int f = 0; f < nrhs; ++f) ua[f] = ub[f] = w.X + (int64_t)f * ndof;
        for (int p = 0; p < o->npairs; ++p) {
            ua[nrhs + p] = w.X + (int64_t)o->pairs[2 * p] * ndof;
            ub[nrhs + p] = w.X + (int64_t)o->pairs[2 * p + 1] * ndof;
        }
        AFD_TRY(launch_sensitivity(m->g, m->kh, m->rho, nf, ua, ub, Sd, s));
        if (host)
            AFD_HIP_TRY(hipMemcpyAsync(S, Sd, (size_t)nf * m->g.nelem * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    AFD_HIP_TRY(hipStreamSynchronize(s));
    const double t3 = now_s();
    int rc = AFD_OK;
    for (int r = 0; r < nrhs; ++r) {
        // AFD_OK only when the true FP64 residual of the returned X meets rtol
        int stt = hsc[r].done == 2 ? AFD_E_BREAKDOWN : (truly_converged(r) ? AFD_OK : AFD_E_NOT_CONVERGED);
        if (bb[r] == 0.0) stt = AFD_OK;
        if (stt != AFD_OK && rc == AFD_OK) rc = stt;
        if (st) {
            st[r].iterations = hsc[r].iters;
            st[r].refinements = refinements;
            st[r].status = stt;
            st[r].coarse_dropped = m->deflate ? m->coarse.dropped : 0;
            st[r].rel_residual_true = bb[r] > 0 ? std::sqrt(rr[r] / bb[r]) : 0.0;
            st[r].t_setup = t1 - t0;
            st[r].t_iter = t2 - t1;
            st[r].t_post = t3 - t2;
        }
    }
    if (rc != AFD_OK)
        set_error(rc == AFD_E_BREAKDOWN
                      ? "solve: breakdown (p.Ap <= 0: singular or indefinite)"
                      : "solve: true residual above rtol (max_iter, restarts or refinement sweeps exhausted)");
    return rc;
}

}  // extern "C"
