// Persistent form of the deflated PCG (Sec. 3.5) for small meshes: one
// workgroup of 1024 threads per right-hand side runs the whole iteration in a
// single launch, with the steps, their order and the stopping rule of the
// launch chain in capi.cpp (Saad et al.'s deflated CG, coarse correction in
// A-DEF2 form).  A right-hand side then occupies one compute unit for the
// whole solve instead of the whole chip for a chain of ~9 dependent launches
// per iteration; the price is that one compute unit's memory parallelism has
// to cover every dependent access of the iteration.
//
// Within the workgroup:
//  * y = A u in two passes: each thread applies rho_e Ke to its elements in
//    the Haar basis and parks the 24 results in an element buffer (24 values
//    per element, component-major so that the stores of a wave are
//    contiguous; it stays in L2); after a barrier each thread gathers, for
//    its nodes, the 8 contributions in a fixed order (A = K_ff extended by the
//    identity on fixed DOFs);
//  * dot products: per-wave shuffle sums, then the 16 wave sums in order;
//  * W^T v: one wave per deflation block, shuffle sums in a fixed order;
//  * E^-1 g: the coarse factor of a single super-block, E^-1 = Linv^T Linv
//    (explicit inverse of the Cholesky factor, padding rows identity, rows of
//    dropped unknowns zero), two triangular products with one wave per row.
// Every summation order is fixed: the result is bitwise reproducible.  Each
// loop's trip count is uniform over the workgroup and every wave reaches the
// end (the iteration stops at max_iter at the latest).
#include "afd_internal.h"
#include "haar_dev.h"

namespace afd {

namespace {

constexpr int NTP = 1024, NWV = NTP / 64;
constexpr int PMAX = 1024;  // largest coarse super-block (and coarse size) of this form

struct PersistP {
    int nx, ny, nz;
    int nnode, nelem;
    const double* rho;
    const uint8_t* nm;
    const double* rinv;
    double ikd[3];
    int deflate;
    int b[3], nb[3];
    double inv_scale;
    int ncoarse, P;
    const double* Linv;
    const double* LinvT;
    const int32_t* perm;   // natural coarse index -> position
    const int32_t* iperm;  // position -> natural (-1: padding)
    const double* F;
    double *X, *R, *Pv, *Q, *Z, *Ye;  // per right-hand side: ndof (Ye: 24 nelem)
    CgScalars* sc;
    double rtol;
    int max_iter;
    int warm;
};

__device__ double wg_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();  // the previous sum's readers are done with red
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWV; ++w) s += red[w];
    return s;
}

// y = A u (and the partial sum of u.y, returned summed over the workgroup)
template <bool CUB>
__device__ double apply(const PersistP& p, const KH<double>& kh, const double* u, double* y, double* ye,
                        double* red) {
    const int sx = p.nx + 1, sxy = (p.nx + 1) * (p.ny + 1);
    for (int e = threadIdx.x; e < p.nelem; e += NTP) {
        const int ex = e % p.nx, ey = (e / p.nx) % p.ny, ez = e / (p.nx * p.ny);
        const int n0 = ex + sx * ey + sxy * ez;
        double fc[2][4][3];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int n = n0 + (a & 1) + sx * ((a >> 1) & 1) + sxy * (a >> 2);
            const uint8_t mk = p.nm[n];
#pragma unroll
            for (int c = 0; c < 3; ++c) fc[a >> 2][a & 3][c] = ((mk >> c) & 1) ? 0.0 : u[3 * n + c];
        }
        double yb[4][3], yt[4][3];
        face_fwd(fc[0]);
        face_fwd(fc[1]);
        element_haar<double, CUB>(kh, p.rho[e], fc[0], fc[1], yb, yt);
        face_inv(yb);
        face_inv(yt);
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) ye[(3 * a + c) * p.nelem + e] = a < 4 ? yb[a][c] : yt[a - 4][c];
    }
    __syncthreads();
    double dot = 0.0;
    for (int n = threadIdx.x; n < p.nnode; n += NTP) {
        const int i = n % sx, j = (n / sx) % (p.ny + 1), k = n / sxy;
        double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const int ex = i - 1 + dx, ey = j - 1 + dy, ez = k - 1 + dz;
                    if (ex < 0 || ex >= p.nx || ey < 0 || ey >= p.ny || ez < 0 || ez >= p.nz) continue;
                    const int e = ex + p.nx * (ey + p.ny * ez), a = (1 - dx) + 2 * (1 - dy) + 4 * (1 - dz);
#pragma unroll
                    for (int c = 0; c < 3; ++c) s[c] += ye[(3 * a + c) * p.nelem + e];
                }
        const uint8_t mk = p.nm[n];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double uc = u[3 * n + c];
            const double v = ((mk >> c) & 1) ? uc : s[c];
            y[3 * n + c] = v;
            dot = fma(uc, v, dot);
        }
    }
    const double r = wg_sum(dot, red);
    return r;  // the barrier in wg_sum also orders y's stores before later readers
}

__device__ __forceinline__ void block_range(const PersistP& p, int ax, int bb, int& lo, int& hi) {
    const int n = ax == 0 ? p.nx : (ax == 1 ? p.ny : p.nz);
    lo = bb * p.b[ax];
    hi = (bb == p.nb[ax] - 1) ? n : lo + p.b[ax] - 1;
}

// gp[perm[6 blk + m]] = sum over B's nodes of w_m . (v - v2) (free DOFs); the
// padding positions of gp stay zero
__device__ void restrict_to(const PersistP& p, const double* v, const double* v2, double* gp) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nblk = p.nb[0] * p.nb[1] * p.nb[2];
    const int sx = p.nx + 1, sxy = (p.nx + 1) * (p.ny + 1);
    for (int blk = wv; blk < nblk; blk += NWV) {
        const int bi[3] = {blk % p.nb[0], (blk / p.nb[0]) % p.nb[1], blk / (p.nb[0] * p.nb[1])};
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) block_range(p, a, bi[a], lo[a], hi[a]);
        const double c0 = 0.5 * (lo[0] + hi[0]), c1 = 0.5 * (lo[1] + hi[1]), c2 = 0.5 * (lo[2] + hi[2]);
        const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
        double m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int q = lane; q < ex * ey * ez; q += 64) {
            const int i = lo[0] + q % ex, j = lo[1] + (q / ex) % ey, k = lo[2] + q / (ex * ey);
            const int n = i + sx * j + sxy * k;
            const uint8_t mk = p.nm[n];
            double u[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) u[c] = ((mk >> c) & 1) ? 0.0 : v[3 * n + c] - (v2 ? v2[3 * n + c] : 0.0);
            const double x = (i - c0) * p.inv_scale, y = (j - c1) * p.inv_scale, z = (k - c2) * p.inv_scale;
            m[0] += u[0];
            m[1] += u[1];
            m[2] += u[2];
            m[3] += -z * u[1] + y * u[2];
            m[4] += z * u[0] - x * u[2];
            m[5] += -y * u[0] + x * u[1];
        }
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double s = m[a];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) s += __shfl_down(s, off, 64);
            if (lane == 0) gp[p.perm[6 * blk + a]] = s;
        }
    }
    __syncthreads();
}

// mu (natural order) = E^-1 g: y = Linv gp, mu_perm = Linv^T y, one wave per
// row (a thread per row, reading the transposed factor coalesced, was slower:
// each row is then a chain of up to P dependent multiply-adds)
__device__ void coarse_solve(const PersistP& p, const double* gp, double* y, double* mu) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = wv; i < p.P; i += NWV) {  // lower triangle: j <= i
        const double* row = p.Linv + (int64_t)i * p.P;
        double s = 0.0;
        for (int j = lane; j <= i; j += 64) s = fma(row[j], gp[j], s);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) y[i] = s;
    }
    __syncthreads();
    for (int i = wv; i < p.P; i += NWV) {  // upper triangle: j >= i
        const double* row = p.LinvT + (int64_t)i * p.P;
        double s = 0.0;
        for (int j = i + lane; j < p.P; j += 64) s = fma(row[j], y[j], s);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_down(s, off, 64);
        const int nat = p.iperm[i];
        if (lane == 0 && nat >= 0) mu[nat] = s;
    }
    __syncthreads();
}

// W mu at node n (zero on fixed DOFs)
__device__ __forceinline__ void prolong_at(const PersistP& p, const double* mu, int n, double w[3]) {
    const int sx = p.nx + 1, sxy = (p.nx + 1) * (p.ny + 1);
    const int pp[3] = {n % sx, (n / sx) % (p.ny + 1), n / sxy};
    int bb[3];
    double x[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int q = pp[a] / p.b[a];
        if (q > p.nb[a] - 1) q = p.nb[a] - 1;
        int lo, hi;
        block_range(p, a, q, lo, hi);
        bb[a] = q;
        x[a] = (pp[a] - 0.5 * (lo + hi)) * p.inv_scale;
    }
    const double* m = mu + 6 * (bb[0] + p.nb[0] * (bb[1] + p.nb[1] * bb[2]));
    const uint8_t mk = p.nm[n];
    w[0] = (mk & 1) ? 0.0 : m[0] + m[4] * x[2] - m[5] * x[1];
    w[1] = (mk & 2) ? 0.0 : m[1] - m[3] * x[2] + m[5] * x[0];
    w[2] = (mk & 4) ? 0.0 : m[2] + m[3] * x[1] - m[4] * x[0];
}

template <bool CUB>
__global__ __launch_bounds__(NTP) void k_dcg_persistent(PersistP p, KH<double> kh) {
    __shared__ double red[NWV];
    __shared__ double gp[PMAX], yv[PMAX], mu[PMAX];
    const int r = blockIdx.x, t = threadIdx.x;
    const int64_t nd = 3 * (int64_t)p.nnode;
    const double* F = p.F + r * nd;
    double *X = p.X + r * nd, *R = p.R + r * nd, *Pv = p.Pv + r * nd, *Q = p.Q + r * nd, *Z = p.Z + r * nd;
    double* ye = p.Ye + (int64_t)r * 24 * p.nelem;
    for (int i = t; i < PMAX; i += NTP) gp[i] = 0.0;
    // ||b||^2
    double acc = 0.0;
    for (int64_t i = t; i < nd; i += NTP) acc = fma(F[i], F[i], acc);
    const double bb = wg_sum(acc, red);
    const double tol2 = p.rtol * p.rtol * bb;
    int iters = 0, done = 0;
    double rr = 0.0;
    // start: x0 = W E^-1 W^T b, or x + W E^-1 W^T (b - A x) from a given x
    if (p.warm) {
        for (int n = t; n < p.nnode; n += NTP) {
            const uint8_t mk = p.nm[n];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((mk >> c) & 1) X[3 * n + c] = 0.0;
        }
        __syncthreads();
        if (p.deflate) {
            apply<CUB>(p, kh, X, Q, ye, red);
            restrict_to(p, F, Q, gp);
        }
    } else {
        for (int64_t i = t; i < nd; i += NTP) X[i] = 0.0;
        __syncthreads();
        if (p.deflate) restrict_to(p, F, nullptr, gp);
    }
    if (p.deflate) {
        coarse_solve(p, gp, yv, mu);
        for (int n = t; n < p.nnode; n += NTP) {
            double w[3];
            prolong_at(p, mu, n, w);
#pragma unroll
            for (int c = 0; c < 3; ++c) X[3 * n + c] += w[c];
        }
        __syncthreads();
    }
    // r = b - A x, z = M^-1 r
    apply<CUB>(p, kh, X, Q, ye, red);
    double rz_acc = 0.0, rr_acc = 0.0;
    for (int n = t; n < p.nnode; n += NTP) {
        const double ri = p.rinv[n];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double rv = F[3 * n + c] - Q[3 * n + c];
            const double zv = ri * p.ikd[c] * rv;
            R[3 * n + c] = rv;
            Z[3 * n + c] = zv;
            rz_acc = fma(rv, zv, rz_acc);
            rr_acc = fma(rv, rv, rr_acc);
        }
    }
    double rz = wg_sum(rz_acc, red);
    rr = wg_sum(rr_acc, red);
    if (bb == 0.0 || rr <= tol2) done = 1;
    double beta = 0.0, pq = 0.0;
    // the first direction: p = z - W E^-1 W^T (A z - r), q = A p
    bool first = true;
    while (!done) {
        if (p.deflate) {
            apply<CUB>(p, kh, Z, Q, ye, red);
            restrict_to(p, Q, R, gp);
            coarse_solve(p, gp, yv, mu);
        }
        for (int n = t; n < p.nnode; n += NTP) {
            double w[3] = {0.0, 0.0, 0.0};
            if (p.deflate) prolong_at(p, mu, n, w);
            const uint8_t mk = p.nm[n];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double v = (first ? 0.0 : beta * Pv[3 * n + c]) + Z[3 * n + c] - w[c];
                Pv[3 * n + c] = ((mk >> c) & 1) ? 0.0 : v;
            }
        }
        first = false;
        __syncthreads();
        pq = apply<CUB>(p, kh, Pv, Q, ye, red);
        if (!(pq > 0.0) || !isfinite(pq)) {
            done = 2;
            break;
        }
        const double alpha = rz / pq;
        rz_acc = 0.0, rr_acc = 0.0;
        for (int n = t; n < p.nnode; n += NTP) {
            const double ri = p.rinv[n];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int64_t i = 3 * (int64_t)n + c;
                X[i] = fma(alpha, Pv[i], X[i]);
                const double rv = fma(-alpha, Q[i], R[i]);
                const double zv = ri * p.ikd[c] * rv;
                R[i] = rv;
                Z[i] = zv;
                rz_acc = fma(rv, zv, rz_acc);
                rr_acc = fma(rv, rv, rr_acc);
            }
        }
        const double rz_new = wg_sum(rz_acc, red);
        rr = wg_sum(rr_acc, red);
        ++iters;
        if (!isfinite(rr)) done = 2;
        else if (rr <= tol2) done = 1;
        else if (iters >= p.max_iter) done = 3;
        beta = rz_new / rz;
        rz = rz_new;
    }
    if (t == 0) {
        CgScalars st = p.sc[r];
        st.iters = iters;
        st.done = done;
        st.rr = rr;
        st.bb = bb;
        st.rz = rz;
        st.pq = pq;
        st.tol2 = tol2;
        st.max_iter = p.max_iter;
        p.sc[r] = st;
    }
}

}  // namespace

bool persistent_fits(const Grid& g, const Blocks& b, bool deflate, int nrhs) {
    if (nrhs < 1 || nrhs > 4 || g.nelem > PERSISTENT_MAX_ELEMS) return false;
    if (!deflate) return true;
    return b.K == 1 && b.P <= PMAX && b.ncoarse <= PMAX;
}

int launch_dcg_persistent(const Grid& g, const Blocks& b, bool deflate, const KeHaar& khd, const double* rho,
                          const uint8_t* nmask, const double* rinv, const double* Linv, const double* LinvT,
                          const int32_t* perm, const int32_t* iperm, int nrhs, const double* F, double* X, double* R,
                          double* P, double* Q, double* Z, double* Ye, CgScalars* sc, double rtol, int max_iter,
                          bool warm, hipStream_t s) {
    if (!persistent_fits(g, b, deflate, nrhs) || max_iter < 1) {
        set_error("persistent solve: mesh or coarse problem too large for one workgroup per right-hand side");
        return AFD_E_INVALID_ARG;
    }
    PersistP p{};
    p.nx = g.nx, p.ny = g.ny, p.nz = g.nz;
    p.nnode = (int)g.nnode, p.nelem = (int)g.nelem;
    p.rho = rho, p.nm = nmask, p.rinv = rinv;
    for (int c = 0; c < 3; ++c) p.ikd[c] = 1.0 / khd.kdiag[c];
    p.deflate = deflate ? 1 : 0;
    for (int a = 0; a < 3; ++a) p.b[a] = b.b[a], p.nb[a] = b.nb[a];
    p.inv_scale = b.inv_scale;
    p.ncoarse = b.ncoarse, p.P = b.P;
    p.Linv = Linv, p.LinvT = LinvT, p.perm = perm, p.iperm = iperm;
    p.F = F, p.X = X, p.R = R, p.Pv = P, p.Q = Q, p.Z = Z, p.Ye = Ye;
    p.sc = sc;
    p.rtol = rtol;
    p.max_iter = max_iter;
    p.warm = warm ? 1 : 0;
    const KH<double> kh = to_kh<double>(khd);
    if (is_cubic(khd)) hipLaunchKernelGGL(k_dcg_persistent<true>, dim3(nrhs), dim3(NTP), 0, s, p, kh);
    else hipLaunchKernelGGL(k_dcg_persistent<false>, dim3(nrhs), dim3(NTP), 0, s, p, kh);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

}  // namespace afd
