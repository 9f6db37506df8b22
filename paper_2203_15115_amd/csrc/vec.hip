// Vector-level kernels of the deflated PCG (Sec. 3.5): Jacobi diagonal formed
// assembly-free, deterministic dot products, CG scalar recurrences kept on the
// device, the fused x/r update, and the deflation operators W^T v / W mu of
// the six rigid-body motions per agglomerated block.
//
// Every reduction is two-stage with a fixed order (per-workgroup partials,
// then one workgroup summing the partials in index order), so results are
// bitwise reproducible; no floating-point atomics are used.
#include <algorithm>
#include <cmath>

#include "afd_internal.h"

namespace afd {

namespace {

constexpr int WG = 256;

__device__ __forceinline__ double wg_reduce(double v, double* sh) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
    const int t = threadIdx.x;
    __syncthreads();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0)
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) s += sh[w];
    return s;  // valid in thread 0
}

// fixed-order sum of n partials by one workgroup (valid in thread 0)
__device__ __forceinline__ double sum_partials(const double* p, int n, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
    return wg_reduce(v, sh);
}

__global__ void k_pack_mask(int64_t nnode, const uint8_t* dm, uint8_t* nm) {
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nnode) return;
    nm[n] = (uint8_t)((dm[3 * n] ? 1 : 0) | (dm[3 * n + 1] ? 2 : 0) | (dm[3 * n + 2] ? 4 : 0));
}

__global__ void k_node_rsum(int nx, int ny, int nz, const double* rho, double* rinv, float* rinv32) {
    const int64_t nnode = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nnode) return;
    const int i = (int)(n % (nx + 1));
    const int j = (int)((n / (nx + 1)) % (ny + 1));
    const int k = (int)(n / ((int64_t)(nx + 1) * (ny + 1)));
    double s = 0.0;
    for (int dz = -1; dz <= 0; ++dz)
        for (int dy = -1; dy <= 0; ++dy)
            for (int dx = -1; dx <= 0; ++dx) {
                const int ex = i + dx, ey = j + dy, ez = k + dz;
                if (ex < 0 || ey < 0 || ez < 0 || ex >= nx || ey >= ny || ez >= nz) continue;
                s += rho[ex + (int64_t)nx * (ey + (int64_t)ny * ez)];
            }
    const double r = 1.0 / s;
    rinv[n] = r;
    rinv32[n] = (float)r;
}

__global__ void k_jacobi_full(int64_t nnode, const double* rinv, const uint8_t* nm, double k0, double k1, double k2,
                              double* d) {
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nnode) return;
    const double kd[3] = {k0, k1, k2};
    for (int c = 0; c < 3; ++c) d[3 * n + c] = ((nm[n] >> c) & 1) ? 1.0 : kd[c] / rinv[n];
}

__global__ void k_dot_partial(int64_t n, const double* x, const double* y, double* part) {
    __shared__ double sh[WG / 64];
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) v += x[i] * y[i];
    v = wg_reduce(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void k_sum(const double* part, int n, double* out) {
    __shared__ double sh[WG / 64];
    double s = sum_partials(part, n, sh);
    if (threadIdx.x == 0) *out = s;
}

// ---- CG scalar recurrences (one workgroup, one rhs per blockIdx.x) -------
// partial layout: [(rhs*2 + which) * npart + i]
__global__ void k_cg_init(CgScalars* sc, const double* part, int npart, double rtol, int max_iter) {
    __shared__ double sh[WG / 64];
    const int r = blockIdx.x;
    double bb = sum_partials(part + (int64_t)(r * 2 + 1) * npart, npart, sh);
    if (threadIdx.x == 0) {
        CgScalars s{};
        s.bb = bb;
        s.tol2 = rtol * rtol * bb;
        s.max_iter = max_iter;
        s.done = (bb == 0.0) ? 1 : 0;
        sc[r] = s;
    }
}

// after the residual of the deflated start: rz, rr
__global__ void k_cg_start(CgScalars* sc, const double* part, int npart) {
    __shared__ double sh[WG / 64];
    const int r = blockIdx.x;
    if (sc[r].done) return;
    double rz = sum_partials(part + (int64_t)(r * 2 + 0) * npart, npart, sh);
    double rr = sum_partials(part + (int64_t)(r * 2 + 1) * npart, npart, sh);
    if (threadIdx.x == 0) {
        sc[r].rz = rz;
        sc[r].rr = rr;
        sc[r].rr0 = rr;
        sc[r].beta = 0.0;
        if (rr <= sc[r].tol2) sc[r].done = 1;
    }
}

__global__ void k_scalar_beta(CgScalars* sc, const double* part, int npart) {
    __shared__ double sh[WG / 64];
    const int r = blockIdx.x;
    if (sc[r].done) return;
    double rz = sum_partials(part + (int64_t)(r * 2 + 0) * npart, npart, sh);
    double rr = sum_partials(part + (int64_t)(r * 2 + 1) * npart, npart, sh);
    if (threadIdx.x == 0) {
        CgScalars s = sc[r];
        s.iters += 1;
        s.rz_new = rz;
        s.rr = rr;
        s.beta = rz / s.rz;
        s.rz = rz;
        if (!isfinite(rr)) s.done = 2;
        else if (rr <= s.tol2) s.done = 1;
        else if (s.iters >= s.max_iter) s.done = 3;
        sc[r] = s;
    }
}

// alpha = r.z / p.q from the p.q partials, then r -= alpha q, z = M^-1 r
// (optional), partials of r.z and r.r, and x += alpha p when X is given (the
// deflated PCG leaves that to k_form_dir, which reads p anyway); flat over
// DOFs so that every array access is a unit-stride stream.  Every workgroup
// sums the p.q partials in the same order and so takes the same alpha;
// workgroup 0 records it (and a breakdown, which every workgroup sees alike).
template <typename T>
__global__ void k_cg_update(int64_t nnode, int64_t ndof, const double* rinv, const float* rinv32,
                            double kd0, double kd1, double kd2, CgScalars* sc, T* X, const T* Pv, T* R,
                            const T* Q, T* Z, double* part, int npart, const double* pqpart, int npq) {
    __shared__ double sh[WG / 64];
    const int r = blockIdx.y;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    // one read of the flag per workgroup: workgroup 0 may set it (breakdown)
    // while others run, and the waves of a workgroup must agree
    __shared__ int done_all;
    if (threadIdx.x == 0) done_all = sc[r].done;
    __syncthreads();
    if (done_all) {
        // the direction kernel of the iteration that set done has run since
        if (lead) sc[r].xdone = 1;
        return;
    }
    __shared__ double pq_all;  // the sum is formed in thread 0; every thread needs it
    const double pq0 = sum_partials(pqpart + (int64_t)(r * 2 + 0) * npq, npq, sh);
    if (threadIdx.x == 0) pq_all = pq0;
    __syncthreads();
    const double pq = pq_all;
    const double rzv = sc[r].rz;
    const bool brk = !(pq > 0.0) || !isfinite(pq) || !isfinite(rzv);
    if (lead) {
        sc[r].pq = pq;
        sc[r].alpha = brk ? 0.0 : rzv / pq;
        if (brk) sc[r].done = 2;  // breakdown: A not SPD on the Krylov space (e.g. no fixed DOFs)
    }
    if (brk) return;
    const T a = (T)(rzv / pq);
    if (X) {  // else x += alpha p is done by k_form_dir
        X += r * ndof;
        Pv += r * ndof;
    }
    R += r * ndof;
    Q += r * ndof;
    if (Z) Z += r * ndof;
    const double ikd[3] = {1.0 / kd0, 1.0 / kd1, 1.0 / kd2};
    double rz = 0.0, rr = 0.0;
    // one element (i < 3 nnode < 2^31, checked at mesh creation)
    auto elem = [&](int i, T rold, T q, double ri) {
        const int c = i - 3 * (i / 3);
        if (X) X[i] = X[i] + a * Pv[i];  // else in k_form_dir
        const T rv = rold - a * q;
        R[i] = rv;
        const double z = ri * ikd[c] * (double)rv;
        if (Z) Z[i] = (T)z;
        rz += (double)rv * z;
        rr += (double)rv * (double)rv;
    };
    auto rinv_of = [&](int i) { return (sizeof(T) == 8) ? rinv[i / 3] : (double)rinv32[i / 3]; };
    const int64_t n = ndof, stride = (int64_t)gridDim.x * WG;  // indices stay 64-bit: i + 4 stride may pass 2^31
    int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    // four elements per step, their loads issued together (one element per
    // step leaves too few loads in flight to cover the memory latency); the
    // elements are still taken in ascending order, so the sums are unchanged
    for (; i + 3 * stride < n; i += 4 * stride) {
        T rv[4], qv[4];
        double ri[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = (int)(i + u * stride);
            rv[u] = R[j];
            qv[u] = Q[j];
            ri[u] = rinv_of(j);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) elem((int)(i + u * stride), rv[u], qv[u], ri[u]);
    }
    for (; i < n; i += stride) elem((int)i, R[i], Q[i], rinv_of((int)i));
    double s0 = wg_reduce(rz, sh);
    double s1 = wg_reduce(rr, sh);
    if (threadIdx.x == 0) {
        part[(int64_t)(r * 2 + 0) * npart + blockIdx.x] = s0;
        part[(int64_t)(r * 2 + 1) * npart + blockIdx.x] = s1;
    }
}

// ---- deflation operators ------------------------------------------------
struct BlkP {
    int nx, ny, nz;
    int b[3], nb[3];
    double inv_scale;
    int ncoarse;
    double rsx, rsxy, rb[3];  // 1/(nx+1), 1/((nx+1)(ny+1)), 1/b: quotients without integer division
};

// floor(a / d) for 0 <= a < 2^31, d >= 1, from rd = 1/d: the double product
// is within one of the quotient, and the two integer tests correct it
__device__ __forceinline__ int quot(int a, int d, double rd) {
    int q = (int)((double)a * rd);
    q -= (int64_t)q * d > a;
    q += (int64_t)(q + 1) * d <= a;
    return q;
}

__device__ __forceinline__ void block_range(const BlkP& p, int ax, int bb, int& lo, int& hi) {
    const int n = ax == 0 ? p.nx : (ax == 1 ? p.ny : p.nz);
    lo = bb * p.b[ax];
    hi = (bb == p.nb[ax] - 1) ? n : lo + p.b[ax] - 1;
}

// block of node n (32-bit node index) and the node's position relative to the
// block centre, scaled by inv_scale
__device__ __forceinline__ void node_block(const BlkP& p, int n, int bb[3], double x[3]) {
    const int sx = p.nx + 1, sxy = (p.nx + 1) * (p.ny + 1);
    const int k = quot(n, sxy, p.rsxy), rem = n - k * sxy, j = quot(rem, sx, p.rsx), i = rem - j * sx;
    const int pp[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int q = quot(pp[a], p.b[a], p.rb[a]);
        if (q > p.nb[a] - 1) q = p.nb[a] - 1;
        int lo, hi;
        block_range(p, a, q, lo, hi);
        bb[a] = q;
        x[a] = (pp[a] - 0.5 * (lo + hi)) * p.inv_scale;
    }
}

// G[r][6*blk+m] = sum over free DOFs of block blk of w_m . V[r]; G = W^T (V - V2)
// (V2 optional).  One wavefront per block (a block has 512-729 nodes), so the
// six sums reduce with shuffles in a fixed order and no barriers.
constexpr int RWG = 64;
// Workgroups are dispatched round-robin over the 8 XCDs (one L2 each): dispatch
// index b -> block so that every XCD gets a contiguous range of blocks, and x
// neighbours, whose node rows share cache lines, share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b % 8, k = b / 8;
    const int base = nb / 8, rem = nb % 8;
    return x * base + min(x, rem) + k;
}
// Optional riders of the restriction inside the CG iteration (each saves a
// launch of its own): the permuted copy of G the coarse solve starts from
// (gperm[r][perm[i]] = G[r][i]), and the CG step's beta/convergence update
// (k_scalar_beta's work) for right-hand side r = blockIdx.x < nrhs, on one
// wavefront of the workgroup (partials summed in a fixed order).
struct RestrictRiders {
    const int32_t* perm = nullptr;
    double* gperm = nullptr;
    int64_t npad = 0;
    CgScalars* sc = nullptr;
    const double* bpart = nullptr;
    int bnpart = 0;
};

__device__ __forceinline__ void beta_step(CgScalars* sc, const double* part, int npart, int r) {
    if (sc[r].done) return;  // same address for the whole wavefront
    double rz = 0.0, rr = 0.0;
    for (int i = threadIdx.x; i < npart; i += RWG) {
        rz += part[(int64_t)(r * 2 + 0) * npart + i];
        rr += part[(int64_t)(r * 2 + 1) * npart + i];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        rz += __shfl_down(rz, off, 64);
        rr += __shfl_down(rr, off, 64);
    }
    if (threadIdx.x == 0) {
        CgScalars st = sc[r];
        st.iters += 1;
        st.rz_new = rz;
        st.rr = rr;
        st.beta = rz / st.rz;
        st.rz = rz;
        if (!isfinite(rr)) st.done = 2;
        else if (rr <= st.tol2) st.done = 1;
        else if (st.iters >= st.max_iter) st.done = 3;
        sc[r] = st;
    }
}

template <typename T>
__global__ __launch_bounds__(RWG) void k_restrict(BlkP p, const uint8_t* nm, int nrhs, int64_t ndof, const T* V,
                                                  const T* V2, double* G, RestrictRiders rd) {
    if (rd.sc && (int)blockIdx.x < nrhs) beta_step(rd.sc, rd.bpart, rd.bnpart, blockIdx.x);
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int bi = blk % p.nb[0], bj = (blk / p.nb[0]) % p.nb[1], bk = blk / (p.nb[0] * p.nb[1]);
    int lo[3], hi[3];
    block_range(p, 0, bi, lo[0], hi[0]);
    block_range(p, 1, bj, lo[1], hi[1]);
    block_range(p, 2, bk, lo[2], hi[2]);
    const double c0 = 0.5 * (lo[0] + hi[0]), c1 = 0.5 * (lo[1] + hi[1]), c2 = 0.5 * (lo[2] + hi[2]);
    const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    const int cnt = ex * ey * ez;
    for (int r = 0; r < nrhs; ++r) {
        const T* v = V + r * ndof;
        const T* v2 = V2 ? V2 + r * ndof : nullptr;
        double m[6] = {0, 0, 0, 0, 0, 0};
        // RU nodes per lane per pass: all their loads are issued before any is
        // used (a block holds 512-729 nodes, 8-12 per lane: one dependent load
        // round per node left this kernel waiting on memory latency); the
        // nodes are still added in ascending order
        constexpr int RU = 4;
        // the lane's node (li, lj, lk) in the block, advanced by RWG nodes per
        // step without integer division (di, dj, dk: RWG in block coordinates)
        const int di = RWG % ex, dj = (RWG / ex) % ey, dk = RWG / (ex * ey);
        int li = threadIdx.x % ex, lj = (threadIdx.x / ex) % ey, lk = threadIdx.x / (ex * ey);
        for (int q0 = threadIdx.x; q0 < cnt; q0 += RU * RWG) {
            double u[RU][3], xyz[RU][3];
            uint8_t mk[RU];
#pragma unroll
            for (int s = 0; s < RU; ++s) {
                const bool in = q0 + s * RWG < cnt;  // past the end: block node 0 again, not added below
                const int i = lo[0] + (in ? li : 0), j = lo[1] + (in ? lj : 0), k = lo[2] + (in ? lk : 0);
                li += di;
                const int ci = li >= ex;
                li -= ci ? ex : 0;
                lj += dj + ci;
                const int cj = lj >= ey;
                lj -= cj ? ey : 0;
                lk += dk + cj;
                const int64_t n = i + (int64_t)(p.nx + 1) * (j + (int64_t)(p.ny + 1) * k);
                mk[s] = nm[n];
                xyz[s][0] = (i - c0) * p.inv_scale;
                xyz[s][1] = (j - c1) * p.inv_scale;
                xyz[s][2] = (k - c2) * p.inv_scale;
#pragma unroll
                for (int c = 0; c < 3; ++c) u[s][c] = (double)v[3 * n + c];
                if (v2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) u[s][c] -= (double)v2[3 * n + c];
                }
            }
#pragma unroll
            for (int s = 0; s < RU; ++s) {
                if (q0 + s * RWG >= cnt) break;
                const double x = xyz[s][0], y = xyz[s][1], z = xyz[s][2];
                const double u0 = (mk[s] & 1) ? 0.0 : u[s][0], u1 = (mk[s] & 2) ? 0.0 : u[s][1],
                             u2 = (mk[s] & 4) ? 0.0 : u[s][2];
                m[0] += u0;
                m[1] += u1;
                m[2] += u2;
                m[3] += -z * u1 + y * u2;
                m[4] += z * u0 - x * u2;
                m[5] += -y * u0 + x * u1;
            }
        }
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double s = m[a];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) s += __shfl_down(s, off, 64);
            if (threadIdx.x == 0) {
                G[(int64_t)r * p.ncoarse + 6 * blk + a] = s;
                if (rd.gperm) rd.gperm[r * rd.npad + rd.perm[6 * blk + a]] = s;
            }
        }
    }
}

// V[r] = W MU[r] (zero on fixed DOFs); or, with color >= 0, the probe vector
// sum over blocks of that 3x3x3 color of motion `mode`.
template <typename T>
__global__ void k_prolong(BlkP p, const uint8_t* nm, int nrhs, int64_t nnode, const double* MU, T* V,
                          int color, int mode) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;  // 3 nnode < 2^31 (checked at mesh creation)
    if (n >= nnode) return;
    const int r = blockIdx.y;
    int bb[3];
    double x[3];
    node_block(p, n, bb, x);
    const uint8_t mk = nm[n];
    double m[6];
    if (color >= 0) {
        const int col = (bb[0] % 3) + 3 * (bb[1] % 3) + 9 * (bb[2] % 3);
        for (int a = 0; a < 6; ++a) m[a] = (col == color && a == mode) ? 1.0 : 0.0;
    } else {
        const double* mu = MU + (int64_t)r * p.ncoarse + 6 * (bb[0] + p.nb[0] * (bb[1] + p.nb[1] * bb[2]));
        for (int a = 0; a < 6; ++a) m[a] = mu[a];
    }
    T* v = V + (int64_t)r * 3 * nnode + 3 * (int64_t)n;
    v[0] = (mk & 1) ? T(0) : (T)(m[0] + m[4] * x[2] - m[5] * x[1]);
    v[1] = (mk & 2) ? T(0) : (T)(m[1] - m[3] * x[2] + m[5] * x[0]);
    v[2] = (mk & 4) ? T(0) : (T)(m[2] + m[3] * x[1] - m[4] * x[0]);
}

// X[r] += W MU[r] on free DOFs, X[r] = 0 on fixed DOFs (the coarse correction
// of a warm start, x0 = x + W E^-1 W^T (b - A x)); MU null: only the masking
// A right-hand side already marked done (a zero b) gets X[r] = 0.
__global__ void k_prolong_add(BlkP p, const uint8_t* nm, int64_t nnode, const double* MU, const CgScalars* sc,
                              double* X) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;  // 3 nnode < 2^31 (checked at mesh creation)
    if (n >= nnode) return;
    const int r = blockIdx.y;
    const uint8_t mk = sc && sc[r].done ? 7 : nm[n];
    double* v = X + (int64_t)r * 3 * nnode + 3 * (int64_t)n;
    double d[3] = {0.0, 0.0, 0.0};
    if (MU) {
        int bb[3];
        double x[3];
        node_block(p, n, bb, x);
        const double* mu = MU + (int64_t)r * p.ncoarse + 6 * (bb[0] + p.nb[0] * (bb[1] + p.nb[1] * bb[2]));
        d[0] = mu[0] + mu[4] * x[2] - mu[5] * x[1];
        d[1] = mu[1] - mu[3] * x[2] + mu[5] * x[0];
        d[2] = mu[2] + mu[3] * x[1] - mu[4] * x[0];
    }
    for (int c = 0; c < 3; ++c) v[c] = ((mk >> c) & 1) ? 0.0 : v[c] + d[c];
}

// p' = beta p + M^-1 r - W mu (zero on fixed DOFs), the direction update of
// the deflated PCG, skipped for converged right-hand sides.  A workgroup
// takes WG consecutive nodes: their 3 WG components of p and r are staged
// through LDS with unit-stride global accesses (a node's three components
// sit 24 bytes apart, so node-per-thread global loads would touch every
// line three times), each thread then updates one node (its block and its
// position in it computed once), and the result leaves through LDS the same
// way.  In place (Pnew == Pold) is allowed.  With X it also applies the
// iteration's x += alpha p (p the old direction, read here anyway), which
// saves k_cg_update a read of p and a read and write of x.
template <typename T>
__global__ __launch_bounds__(WG) void k_form_dir(BlkP p, const uint8_t* nm, int64_t nnode, const CgScalars* sc,
                                                 const double* MU, const T* Pold, const T* R, const double* rinv,
                                                 const float* rinv32, double ikd0, double ikd1, double ikd2,
                                                 T* Pnew, T* X) {
    __shared__ T sp[3 * WG], sr[3 * WG];
    const int r = blockIdx.y;
    // X: x += alpha p_old, also in the iteration whose restriction set done
    // (once: the next alpha kernel sets xdone); p' only while running
    const bool dn = sc[r].done != 0;
    const bool doX = X != nullptr && !(dn && sc[r].xdone);
    if (dn && !doX) return;
    const int t = threadIdx.x;
    const int64_t n0 = (int64_t)blockIdx.x * WG;  // 3 nnode < 2^31 (checked at mesh creation)
    const int cnt = (int)min((int64_t)WG, nnode - n0);
    const int nv = 3 * cnt;
    const int64_t base = (int64_t)r * 3 * nnode + 3 * n0;
    const T a = (T)sc[r].alpha;
    // nv <= 3 WG: three unrolled steps, so that their loads are in flight together
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int e = t + k * WG;
        if (e < nv) {
            const T pv = Pold[base + e];
            if (doX) X[base + e] = X[base + e] + a * pv;
            sp[e] = pv;
            if (!dn) sr[e] = R[base + e];
        }
    }
    if (dn) return;  // the same for the whole workgroup
    __syncthreads();
    if (t < cnt) {
        const int n = (int)(n0 + t);
        const double beta = sc[r].beta;
        double w[3] = {0.0, 0.0, 0.0};
        if (MU) {
            int bb[3];
            double x[3];
            node_block(p, n, bb, x);
            const double* m = MU + (int64_t)r * p.ncoarse + 6 * (bb[0] + p.nb[0] * (bb[1] + p.nb[1] * bb[2]));
            w[0] = m[0] + m[4] * x[2] - m[5] * x[1];
            w[1] = m[1] - m[3] * x[2] + m[5] * x[0];
            w[2] = m[2] + m[3] * x[1] - m[4] * x[0];
        }
        const double ri = rinv ? rinv[n] : (double)rinv32[n];
        // M^-1 r formed exactly as in k_cg_update and k_precond (the host's
        // 1 / kd is the same correctly rounded quotient they form)
        const double ikd[3] = {ikd0, ikd1, ikd2};
        const uint8_t mk = nm[n];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = beta * (double)sp[3 * t + c] + ri * ikd[c] * (double)sr[3 * t + c] - w[c];
            sp[3 * t + c] = ((mk >> c) & 1) ? T(0) : (T)v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int e = t + k * WG;
        if (e < nv) Pnew[base + e] = sp[e];
    }
}

__global__ void k_copy(int64_t n, const double* a, double* b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}
template <typename T>
__global__ void k_fill(int64_t n, T v, T* a) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}


template <typename T>
__global__ void k_dot_partial_t(int64_t n, const T* x, double* part) {
    __shared__ double sh[WG / 64];
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG)
        v += (double)x[i] * (double)x[i];
    v = wg_reduce(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// z = M^-1 r (Jacobi), zero on fixed DOFs through r
template <typename T>
__global__ void k_precond(int64_t nnode, int64_t ndof, const double* rinv, const float* rinv32, double kd0,
                          double kd1, double kd2, const T* R, T* Z) {
    const int r = blockIdx.y;
    const double ikd[3] = {1.0 / kd0, 1.0 / kd1, 1.0 / kd2};
    for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < ndof; i += (int64_t)gridDim.x * WG) {
        const int64_t n = i / 3;
        const int c = (int)(i - 3 * n);
        const double ri = rinv ? rinv[n] : (double)rinv32[n];
        Z[r * ndof + i] = (T)(ri * ikd[c] * (double)R[r * ndof + i]);
    }
}

// outer refinement: rr from partials; converged or scale = ||r||
__global__ void k_outer_norm(CgScalars* sc, const double* part, int npart) {
    __shared__ double sh[WG / 64];
    const int r = blockIdx.x;
    if (sc[r].done) return;
    double rr = sum_partials(part + (int64_t)(r * 2 + 1) * npart, npart, sh);
    if (threadIdx.x == 0) {
        sc[r].rr = rr;
        if (!isfinite(rr)) sc[r].done = 2;
        else if (rr <= sc[r].tol2) sc[r].done = 1;
        else if (sc[r].iters >= sc[r].max_iter) sc[r].done = 3;
        else {
            sc[r].alpha = sqrt(rr);
            sc[r].iters += 1;
        }
    }
}

__global__ void k_to_f32_scaled(int64_t ndof, const double* R, const CgScalars* sc, float* Rf) {
    const int r = blockIdx.y;
    const bool dn = sc[r].done != 0;
    const double inv = dn ? 0.0 : 1.0 / sc[r].alpha;
    for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < ndof; i += (int64_t)gridDim.x * WG)
        Rf[r * ndof + i] = dn ? 0.0f : (float)(R[r * ndof + i] * inv);
}

__global__ void k_axpy_refine(int64_t ndof, const CgScalars* sc, const float* D, double* X) {
    const int r = blockIdx.y;
    if (sc[r].done) return;
    const double a = sc[r].alpha;
    for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < ndof; i += (int64_t)gridDim.x * WG)
        X[r * ndof + i] += a * (double)D[r * ndof + i];
}

BlkP blkp(const Grid& g, const Blocks& b) {
    BlkP p;
    p.nx = g.nx;
    p.ny = g.ny;
    p.nz = g.nz;
    for (int a = 0; a < 3; ++a) {
        p.b[a] = b.b[a];
        p.nb[a] = b.nb[a];
    }
    p.inv_scale = b.inv_scale;
    p.ncoarse = b.ncoarse;
    p.rsx = 1.0 / (g.nx + 1);
    p.rsxy = 1.0 / ((double)(g.nx + 1) * (g.ny + 1));
    for (int a = 0; a < 3; ++a) p.rb[a] = 1.0 / std::max(b.b[a], 1);
    return p;
}

inline unsigned nblocks(int64_t n, int per = WG) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int launch_pack_mask(const Grid& g, const uint8_t* dofmask, uint8_t* nmask, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_mask, dim3(nblocks(g.nnode)), dim3(WG), 0, s, g.nnode, dofmask, nmask);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_node_rsum(const Grid& g, const double* rho, double* rinv, float* rinv32, hipStream_t s) {
    hipLaunchKernelGGL(k_node_rsum, dim3(nblocks(g.nnode)), dim3(WG), 0, s, g.nx, g.ny, g.nz, rho, rinv, rinv32);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_jacobi_full(const Grid& g, const double* rinv, const uint8_t* nmask, const KeHaar& kh, double* d,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_full, dim3(nblocks(g.nnode)), dim3(WG), 0, s, g.nnode, rinv, nmask, kh.kdiag[0],
                       kh.kdiag[1], kh.kdiag[2], d);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_dot(int64_t n, const double* x, const double* y, double* partial, int npart, double* out,
               hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(npart), dim3(WG), 0, s, n, x, y, partial);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(WG), 0, s, partial, npart, out);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

// bb partials: slot 1 of each rhs holds f.f
int launch_dot_rhs(int64_t ndof, int nrhs, const double* F, double* partial, int npart, hipStream_t s) {
    for (int r = 0; r < nrhs; ++r)
        hipLaunchKernelGGL(k_dot_partial, dim3(npart), dim3(WG), 0, s, ndof, F + r * ndof, F + r * ndof,
                           partial + (int64_t)(r * 2 + 1) * npart);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_cg_init(CgScalars* sc, int nrhs, const double* part, int npart, double rtol, int max_iter,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init, dim3(nrhs), dim3(WG), 0, s, sc, part, npart, rtol, max_iter);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}
int launch_cg_start(CgScalars* sc, int nrhs, const double* part, int npart, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_start, dim3(nrhs), dim3(WG), 0, s, sc, part, npart);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}
int launch_scalar_beta(CgScalars* sc, int nrhs, const double* part, int npart, hipStream_t s) {
    hipLaunchKernelGGL(k_scalar_beta, dim3(nrhs), dim3(WG), 0, s, sc, part, npart);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_cg_update(const Grid& g, const KeHaar& kh, const double* rinv, CgScalars* sc, int nrhs, double* X,
                     const double* Pv, double* R, const double* Q, double* Z, double* partial, int npart,
                     const double* pqpart, int npq, hipStream_t s) {
    hipLaunchKernelGGL((k_cg_update<double>), dim3(npart, nrhs), dim3(WG), 0, s, g.nnode, g.ndof, rinv,
                       (const float*)nullptr, kh.kdiag[0], kh.kdiag[1], kh.kdiag[2], sc, X, Pv, R, Q, Z, partial,
                       npart, pqpart, npq);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_cg_update_f32(const Grid& g, const KeHaar& kh, const float* rinv32, CgScalars* sc, int nrhs, float* X,
                         const float* Pv, float* R, const float* Q, float* Z, double* partial, int npart,
                         const double* pqpart, int npq, hipStream_t s) {
    hipLaunchKernelGGL((k_cg_update<float>), dim3(npart, nrhs), dim3(WG), 0, s, g.nnode, g.ndof,
                       (const double*)nullptr, rinv32, kh.kdiag[0], kh.kdiag[1], kh.kdiag[2], sc, X, Pv, R, Q, Z,
                       partial, npart, pqpart, npq);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_restrict(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* V, double* G,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_restrict<double>), dim3(b.nblk), dim3(RWG), 0, s, blkp(g, b), nmask, nrhs, g.ndof, V,
                       (const double*)nullptr, G, RestrictRiders{});
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_prolong(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* MU, double* V,
                   hipStream_t s) {
    hipLaunchKernelGGL((k_prolong<double>), dim3(nblocks(g.nnode), nrhs), dim3(WG), 0, s, blkp(g, b), nmask, nrhs,
                       g.nnode, MU, V, -1, 0);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_prolong_add(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* MU,
                       const CgScalars* sc, double* X, hipStream_t s) {
    hipLaunchKernelGGL(k_prolong_add, dim3(nblocks(g.nnode), nrhs), dim3(WG), 0, s, blkp(g, b), nmask, g.nnode, MU,
                       sc, X);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_form_dir(const Grid& g, const Blocks& b, const uint8_t* nmask, const KeHaar& kh, const CgScalars* sc,
                    int nrhs, const double* MU, const double* rinv, const double* Pold, const double* R,
                    double* Pnew, double* X, hipStream_t s) {
    hipLaunchKernelGGL((k_form_dir<double>), dim3(nblocks(g.nnode), nrhs), dim3(WG), 0, s, blkp(g, b), nmask, g.nnode,
                       sc, MU, Pold, R, rinv, (const float*)nullptr, 1.0 / kh.kdiag[0], 1.0 / kh.kdiag[1],
                       1.0 / kh.kdiag[2], Pnew, X);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_form_dir_f32(const Grid& g, const Blocks& b, const uint8_t* nmask, const KeHaar& kh,
                        const CgScalars* sc, int nrhs, const double* MU, const float* rinv32, const float* Pold,
                        const float* R, float* Pnew, float* X, hipStream_t s) {
    hipLaunchKernelGGL((k_form_dir<float>), dim3(nblocks(g.nnode), nrhs), dim3(WG), 0, s, blkp(g, b), nmask, g.nnode,
                       sc, MU, Pold, R, (const double*)nullptr, rinv32, 1.0 / kh.kdiag[0], 1.0 / kh.kdiag[1],
                       1.0 / kh.kdiag[2], Pnew, X);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_probe_vector(const Grid& g, const Blocks& b, const uint8_t* nmask, int color, int mode, double* V,
                        hipStream_t s) {
    hipLaunchKernelGGL((k_prolong<double>), dim3(nblocks(g.nnode), 1), dim3(WG), 0, s, blkp(g, b), nmask, 1,
                       g.nnode, (const double*)nullptr, V, color, mode);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_copy_f64(int64_t n, const double* a, double* b, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(1024), dim3(WG), 0, s, n, a, b);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}
int launch_fill_f64(int64_t n, double v, double* a, hipStream_t s) {
    hipLaunchKernelGGL((k_fill<double>), dim3(1024), dim3(WG), 0, s, n, v, a);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}
int launch_fill_f32(int64_t n, float v, float* a, hipStream_t s) {
    hipLaunchKernelGGL((k_fill<float>), dim3(1024), dim3(WG), 0, s, n, v, a);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_restrict_diff(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* V,
                         const double* V2, double* G, hipStream_t s, const int32_t* perm, double* gperm, int64_t npad,
                         CgScalars* sc, const double* bpart, int bnpart) {
    RestrictRiders rd;
    rd.perm = perm, rd.gperm = gperm, rd.npad = npad, rd.sc = sc, rd.bpart = bpart, rd.bnpart = bnpart;
    if (sc && b.nblk < nrhs) {
        set_error("restrict: fewer blocks than right-hand sides for the fused scalar update");
        return AFD_E_INVALID_ARG;
    }
    hipLaunchKernelGGL((k_restrict<double>), dim3(b.nblk), dim3(RWG), 0, s, blkp(g, b), nmask, nrhs, g.ndof, V, V2, G,
                       rd);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_restrict_diff_f32(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const float* V,
                             const float* V2, double* G, hipStream_t s, const int32_t* perm, double* gperm,
                             int64_t npad, CgScalars* sc, const double* bpart, int bnpart) {
    RestrictRiders rd;
    rd.perm = perm, rd.gperm = gperm, rd.npad = npad, rd.sc = sc, rd.bpart = bpart, rd.bnpart = bnpart;
    if (sc && b.nblk < nrhs) {
        set_error("restrict: fewer blocks than right-hand sides for the fused scalar update");
        return AFD_E_INVALID_ARG;
    }
    hipLaunchKernelGGL((k_restrict<float>), dim3(b.nblk), dim3(RWG), 0, s, blkp(g, b), nmask, nrhs, g.ndof, V, V2, G,
                       rd);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_restrict_f32(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const float* V, double* G,
                        hipStream_t s) {
    hipLaunchKernelGGL((k_restrict<float>), dim3(b.nblk), dim3(RWG), 0, s, blkp(g, b), nmask, nrhs, g.ndof, V,
                       (const float*)nullptr, G, RestrictRiders{});
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_prolong_f32(const Grid& g, const Blocks& b, const uint8_t* nmask, int nrhs, const double* MU, float* V,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_prolong<float>), dim3(nblocks(g.nnode), nrhs), dim3(WG), 0, s, blkp(g, b), nmask, nrhs,
                       g.nnode, MU, V, -1, 0);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_dot_rhs_f32(int64_t ndof, int nrhs, const float* F, double* partial, int npart, hipStream_t s) {
    for (int r = 0; r < nrhs; ++r)
        hipLaunchKernelGGL((k_dot_partial_t<float>), dim3(npart), dim3(WG), 0, s, ndof, F + r * ndof,
                           partial + (int64_t)(r * 2 + 1) * npart);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_precond(const Grid& g, const KeHaar& kh, const double* rinv, int nrhs, const double* R, double* Z,
                   hipStream_t s) {
    hipLaunchKernelGGL((k_precond<double>), dim3(VEC_NPART, nrhs), dim3(WG), 0, s, g.nnode, g.ndof, rinv,
                       (const float*)nullptr, kh.kdiag[0], kh.kdiag[1], kh.kdiag[2], R, Z);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_precond_f32(const Grid& g, const KeHaar& kh, const float* rinv32, int nrhs, const float* R, float* Z,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_precond<float>), dim3(VEC_NPART, nrhs), dim3(WG), 0, s, g.nnode, g.ndof,
                       (const double*)nullptr, rinv32, kh.kdiag[0], kh.kdiag[1], kh.kdiag[2], R, Z);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_outer_norm(CgScalars* outer, int nrhs, const double* part, int npart, hipStream_t s) {
    hipLaunchKernelGGL(k_outer_norm, dim3(nrhs), dim3(WG), 0, s, outer, part, npart);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_to_f32_scaled(int64_t ndof, int nrhs, const double* R, const CgScalars* outer, float* Rf,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32_scaled, dim3(VEC_NPART, nrhs), dim3(WG), 0, s, ndof, R, outer, Rf);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_axpy_refine(int64_t ndof, int nrhs, const CgScalars* outer, const float* D, double* X, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_refine, dim3(VEC_NPART, nrhs), dim3(WG), 0, s, ndof, outer, D, X);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

}  // namespace afd
