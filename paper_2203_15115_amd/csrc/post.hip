// Post-processing of a solve: per-element energies (the element term
// u^T K^e u of Eq. 3.5, the element-sensitivity route of Sec. 3.1) and the
// topology extracted at a volume fraction by ranking a sensitivity field
// (Eq. 3.6 with the cutting value set by the target volume, Sec. 3.2).
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "afd_internal.h"
#include "voxel_dev.h"

namespace afd {

namespace {

constexpr int MAXF = 16;

struct SensP {
    int nx, ny, nz;
    int nfields;
    const double* ua[MAXF];
    const double* ub[MAXF];
    KeHaar kh;
};

// S[f][e] = rho_e * u_e^T Ke v_e = rho_e * (T u_e)^T Khat (T v_e)
__global__ void k_sensitivity(SensP p, const double* rho, double* S) {
    // 32-bit element and node indices (the host checks n_elem and n_node < 2^31)
    const int nE = p.nx * p.ny * p.nz;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const int ex = e % p.nx, exy = e / p.nx, ey = exy % p.ny, ez = exy / p.ny;
    const int sy = p.nx + 1, sz = (p.nx + 1) * (p.ny + 1);
    int nd[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) nd[a] = (ex + (a & 1)) + sy * (ey + ((a >> 1) & 1)) + sz * (ez + (a >> 2));
    const double r = rho[e];
    auto gather = [&](const double* x, double w[8][3]) {
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) w[a][c] = x[3 * (int64_t)nd[a] + c];
    };
    for (int f = 0; f < p.nfields; ++f) {
        double u[8][3], v[8][3];
        gather(p.ua[f], u);
        haar_fwd(u);
        if (p.ub[f] == p.ua[f]) {  // self energy: one gather and one transform
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) v[a][c] = u[a][c];
        } else {
            gather(p.ub[f], v);
            haar_fwd(v);
        }
        double s = 0.0;
#pragma unroll
        for (int al = 1; al < 8; ++al)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double acc = p.kh.dg[i][al] * v[al][i];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (j == i) continue;
                    const int k = 3 - i - j;
                    const int bi = (al >> i) & 1, bj = (al >> j) & 1, bk = (al >> k) & 1;
                    if (bi == bj) continue;
                    acc = fma(bi ? p.kh.cl[k][bk] : p.kh.cm[k][bk], v[al ^ (1 << i) ^ (1 << j)][j], acc);
                }
                s = fma(u[al][i], acc, s);
            }
        S[(int64_t)f * nE + e] = r * s;
    }
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sort (8-bit digits) of 64-bit keys with int32 payloads.
constexpr int RS_T = 256;     // threads
constexpr int RS_R = 8;       // rounds (keys per thread)
constexpr int RS_TILE = RS_T * RS_R;

// Orders doubles descending as an unsigned key ascending.  -0.0 is keyed as
// +0.0 (equal numbers rank by the next key, not by their bit patterns).
__device__ __forceinline__ uint64_t desc_key(double v) {
    if (v == 0.0) v = 0.0;
    uint64_t b = (uint64_t)__double_as_longlong(v);
    b = (b >> 63) ? ~b : (b | 0x8000000000000000ull);  // ascending order of the double
    return ~b;                                         // descending
}

// keys of s in element order, payload = element index
__global__ void k_make_keys(int64_t n, const double* s, uint64_t* key, int32_t* idx) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = desc_key(s[i]);
    idx[i] = (int32_t)i;
}

// secondary (tie) keys in element order: sorted first, so that the stable
// passes over s keep (tie, index) order among equal values
__global__ void k_make_tie_keys(int64_t n, const int32_t* tie, uint64_t* key, int32_t* idx) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint64_t)(uint32_t)tie[i];
    idx[i] = (int32_t)i;
}

// keys of s in the current order of the payload
__global__ void k_make_keys_perm(int64_t n, const double* s, const int32_t* idx, uint64_t* key) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = desc_key(s[idx[i]]);
}

__global__ void k_hist(int64_t n, const uint64_t* key, int shift, uint32_t* hist, int ntiles) {
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_R; ++r) {
        const int64_t i = base + r * RS_T + t;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * ntiles + blockIdx.x] = h[t];
}

// per digit: exclusive prefix over tiles (in place) and the digit total
__global__ void k_scan_tiles(uint32_t* hist, int ntiles, uint32_t* dtot) {
    __shared__ uint32_t sh[256];
    const int d = blockIdx.x, t = threadIdx.x;
    uint32_t* h = hist + (int64_t)d * ntiles;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += 256) {
        const uint32_t v = (b0 + t < ntiles) ? h[b0 + t] : 0u;
        sh[t] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele
            uint32_t a = (t >= off) ? sh[t - off] : 0u;
            __syncthreads();
            sh[t] += a;
            __syncthreads();
        }
        if (b0 + t < ntiles) h[b0 + t] = carry + sh[t] - v;
        carry += sh[255];
        __syncthreads();
    }
    if (t == 0) dtot[d] = carry;
}

__global__ void k_scan_digits(uint32_t* dtot) {
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int d = 0; d < 256; ++d) {
            const uint32_t v = dtot[d];
            dtot[d] = run;
            run += v;
        }
    }
}

__global__ void k_scatter(int64_t n, const uint64_t* kin, const int32_t* iin, uint64_t* kout, int32_t* iout,
                          int shift, const uint32_t* hist, int ntiles, const uint32_t* dbase) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[RS_T / 64][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    run[t] = dbase[t] + hist[(int64_t)t * ntiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_R; ++r) {
        for (int q = 0; q < RS_T / 64; ++q) wc[q][t] = 0;
        __syncthreads();
        const int64_t i = base + r * RS_T + t;
        const bool valid = i < n;
        uint64_t k = valid ? kin[i] : 0;
        const int d = (int)((k >> shift) & 255);
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bs = __ballot(valid && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? bs : ~bs;
        }
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d] + rank;
            for (int q = 0; q < w; ++q) off += wc[q][d];
            kout[off] = k;
            iout[off] = iin[i];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int q = 0; q < RS_T / 64; ++q) add += wc[q][t];
        run[t] += add;
        __syncthreads();
    }
}

// Casting projection (Sec. 3.7): a running maximum along every line of
// elements parallel to the casting axis, from each far end toward the parting
// plane (elements j >= parting from the last one down, j < parting from the
// first one up).  Maxima are exact: any evaluation order gives the same value
// (a zero is stored as +0.0, whichever signed zero fmax returned).
// Along y and z (strided lines): a workgroup takes 64 consecutive lines (one
// wavefront reads 64 consecutive elements per step) and cuts each side of
// every line into 4 chunks, one wavefront per chunk: the chunk maxima go
// through LDS, then each chunk runs its maximum from the carry of the chunks
// farther out (every element is read twice, written once; the lines alone
// are too few to fill the GPU).
constexpr int CCH = 4;
__global__ __launch_bounds__(256) void k_cast_yz(int nx, int ny, int nz, int axis, int parting, const double* phi,
                                                 double* out) {
    __shared__ double cmax[2][CCH][64];
    const int li = threadIdx.x & 63, c = threadIdx.x >> 6;
    const int L = blockIdx.x * 64 + li;
    int64_t base, stride;
    int n, lines;
    if (axis == 1) {
        lines = nx * nz, n = ny, stride = nx;
        base = (int64_t)(L % nx) + (int64_t)nx * ny * (L / nx);
    } else {
        lines = nx * ny, n = nz, stride = (int64_t)nx * ny, base = L;
    }
    const bool valid = L < lines;
    // this chunk of each side: side + runs j = hi..lo downward, side - j = lo2..hi2 upward
    const int cl = (n - parting + CCH - 1) / CCH, hi = n - 1 - c * cl, lo = max(parting, hi - cl + 1);
    const int cl2 = (parting + CCH - 1) / CCH, lo2 = c * cl2, hi2 = min(parting - 1, lo2 + cl2 - 1);
    double m = -INFINITY, m2 = -INFINITY;
    if (valid) {
        for (int j = hi; j >= lo; --j) m = fmax(m, phi[base + j * stride]);
        for (int j = lo2; j <= hi2; ++j) m2 = fmax(m2, phi[base + j * stride]);
    }
    cmax[0][c][li] = m;
    cmax[1][c][li] = m2;
    __syncthreads();
    if (!valid) return;
    double run = -INFINITY, run2 = -INFINITY;
    for (int k = 0; k < c; ++k) {
        run = fmax(run, cmax[0][k][li]);
        run2 = fmax(run2, cmax[1][k][li]);
    }
    for (int j = hi; j >= lo; --j) {
        run = fmax(run, phi[base + j * stride]);
        out[base + j * stride] = run == 0.0 ? 0.0 : run;
    }
    for (int j = lo2; j <= hi2; ++j) {
        run2 = fmax(run2, phi[base + j * stride]);
        out[base + j * stride] = run2 == 0.0 ? 0.0 : run2;
    }
}

// Along x (contiguous lines) one wavefront per line: 64 consecutive elements
// per step, a running maximum across the lanes by shuffles (log2 64 steps) on
// top of the carry from the previous step.
__global__ void k_cast_x(int nx, int lines, int parting, const double* phi, double* out) {
    const int lane = threadIdx.x & 63;
    const int L = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (L >= lines) return;
    const int64_t base = (int64_t)nx * L;
    double carry = -INFINITY;
    for (int j0 = nx - 1; j0 >= parting; j0 -= 64) {  // side j >= parting, from the far end
        const int j = j0 - lane;
        double v = j >= parting ? phi[base + j] : -INFINITY;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double o = __shfl_up(v, off, 64);
            if (lane >= off) v = fmax(v, o);
        }
        v = fmax(v, carry);
        if (j >= parting) out[base + j] = v == 0.0 ? 0.0 : v;
        carry = __shfl(v, 63, 64);
    }
    carry = -INFINITY;
    for (int j0 = 0; j0 < parting; j0 += 64) {  // side j < parting, from the first element
        const int j = j0 + lane;
        double v = j < parting ? phi[base + j] : -INFINITY;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double o = __shfl_up(v, off, 64);
            if (lane >= off) v = fmax(v, o);
        }
        v = fmax(v, carry);
        if (j < parting) out[base + j] = v == 0.0 ? 0.0 : v;
        carry = __shfl(v, 63, 64);
    }
}

// distance of every element from the parting plane along the casting axis:
// j - parting for j >= parting, parting - 1 - j below (the tie key that cuts
// plateaus of the projected field nearer the plane first)
__global__ void k_parting_distance(int nx, int ny, int nz, int axis, int parting, int32_t* dist) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)nx * ny * nz) return;
    const int64_t sxy = (int64_t)nx * ny;
    const int j = axis == 0 ? (int)(e % nx) : (axis == 1 ? (int)((e % sxy) / nx) : (int)(e / sxy));
    dist[e] = j >= parting ? j - parting : parting - 1 - j;
}

// ---- p-norm von Mises stress (Eq. 3.3, 3.23) --------------------------
// Element stress at the voxel centre (centroid_stress).
struct StressP {
    int nx, ny, nz;
    int nrhs;
    int64_t ndof;
    double inv4h[3];
    double lam, mu, p;
    const double* U;     // [nrhs][ndof]
    const double* rho;
    double* vm;          // [nrhs][nE] or null
    double* part;        // [nrhs][gridDim.x]: per-workgroup sums of vm^p
    double* T;           // [nrhs][6][nE] or null: rho vm^(p-2) D V sigma (adjoint terms)
};

__global__ __launch_bounds__(256) void k_stress(StressP p) {
    __shared__ double red[256 / 64];
    const int nE = p.nx * p.ny * p.nz;  // < 2^31 (checked on the host)
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    double vp = 0.0;
    if (e < nE) {
        const int ex = e % p.nx, exy = e / p.nx, ey = exy % p.ny, ez = exy / p.ny;
        const int sy = p.nx + 1, sz = (p.nx + 1) * (p.ny + 1);
        const double* u0 = p.U + (int64_t)r * p.ndof;
        double h[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int64_t nd = (ex + (a & 1)) + sy * (ey + ((a >> 1) & 1)) + (int64_t)sz * (ez + (a >> 2));
#pragma unroll
            for (int c = 0; c < 3; ++c) h[a][c] = u0[3 * nd + c];
        }
        haar_fwd(h);
        const double rho = p.rho[e];
        double sg[6];
        centroid_stress(h, p.inv4h, p.lam, p.mu, rho, sg);
        const double sxx = sg[0], syy = sg[1], szz = sg[2], tyz = sg[3], txz = sg[4], txy = sg[5];
        const double q = sxx * sxx + syy * syy + szz * szz - sxx * syy - syy * szz - szz * sxx +
                         3.0 * (tyz * tyz + txz * txz + txy * txy);
        const double vm = sqrt(fmax(q, 0.0));
        vp = pow(vm, p.p);
        if (p.vm) p.vm[(int64_t)r * nE + e] = vm;
        if (p.T) {
            const double w = rho * pow(vm, p.p - 2.0);
            const double a0 = sxx - 0.5 * (syy + szz), a1 = syy - 0.5 * (sxx + szz), a2 = szz - 0.5 * (sxx + syy);
            const double ta = p.lam * (a0 + a1 + a2);
            double* T = p.T + (int64_t)r * 6 * nE + e;
            T[0] = w * (ta + 2.0 * p.mu * a0);
            T[(int64_t)nE] = w * (ta + 2.0 * p.mu * a1);
            T[2 * (int64_t)nE] = w * (ta + 2.0 * p.mu * a2);
            T[3 * (int64_t)nE] = w * p.mu * 3.0 * tyz;
            T[4 * (int64_t)nE] = w * p.mu * 3.0 * txz;
            T[5 * (int64_t)nE] = w * p.mu * 3.0 * txy;
        }
    }
    // fixed-order workgroup sum of vm^p
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) vp += __shfl_down(vp, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = vp;
    __syncthreads();
    if (threadIdx.x == 0) p.part[(int64_t)r * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// B[r] at node n: scale * sum over the node's elements of B_c,a^T t_e (a the
// node's corner of element e), zero on fixed DOFs: the adjoint right-hand side
__global__ void k_stress_rhs(StressP p, const uint8_t* nmask, double scale, double* B) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int nn = (nx + 1) * (ny + 1) * (nz + 1);
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int r = blockIdx.y;
    const int nE = nx * ny * nz;
    const int i = n % (nx + 1), ij = n / (nx + 1), j = ij % (ny + 1), k = ij / (ny + 1);
    const double* T = p.T + (int64_t)r * 6 * nE;
    double f[3] = {0.0, 0.0, 0.0};
    for (int dz = 0; dz < 2; ++dz) {
        const int ez = k - 1 + dz;
        if (ez < 0 || ez >= nz) continue;
        for (int dy = 0; dy < 2; ++dy) {
            const int ey = j - 1 + dy;
            if (ey < 0 || ey >= ny) continue;
            for (int dx = 0; dx < 2; ++dx) {
                const int ex = i - 1 + dx;
                if (ex < 0 || ex >= nx) continue;
                const int e = ex + nx * (ey + ny * ez);
                // the node is corner (1 - dx, 1 - dy, 1 - dz) of element e: sign +1 on the far side
                const double gx = (dx ? -1.0 : 1.0) * p.inv4h[0], gy = (dy ? -1.0 : 1.0) * p.inv4h[1],
                             gz = (dz ? -1.0 : 1.0) * p.inv4h[2];
                const double txx = T[e], tyy = T[(int64_t)nE + e], tzz = T[2 * (int64_t)nE + e],
                             tyz = T[3 * (int64_t)nE + e], txz = T[4 * (int64_t)nE + e], txy = T[5 * (int64_t)nE + e];
                f[0] += gx * txx + gy * txy + gz * txz;
                f[1] += gx * txy + gy * tyy + gz * tyz;
                f[2] += gx * txz + gy * tyz + gz * tzz;
            }
        }
    }
    const uint8_t m = nmask[n];
    double* b = B + (int64_t)r * p.ndof + 3 * (int64_t)n;
#pragma unroll
    for (int c = 0; c < 3; ++c) b[c] = ((m >> c) & 1) ? 0.0 : scale * f[c];
}

// ---- the augmented topological level set (Eq. 3.17-3.18) -------------
// out = sum_t coef[t] * (sum over the rows of group t of its fields), with
// the terms and the rows added in order and no fused multiply-add, so that the
// result is the same double as the plain expression evaluated left to right
constexpr int MAX_TERMS = 4;
struct CombineP {
    const double* f[MAX_TERMS];  // group t: rows f[t][r * n + e], r < rows[t]
    int rows[MAX_TERMS];
    double coef[MAX_TERMS];
    int nterms;
};
__global__ void k_combine(int64_t n, CombineP p, double* out) {
#pragma clang fp contract(off)
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    double acc = 0.0;
    for (int t = 0; t < p.nterms; ++t) {
        double s = p.f[t][e];
        for (int r = 1; r < p.rows[t]; ++r) s = s + p.f[t][(int64_t)r * n + e];
        const double term = p.coef[t] * s;
        acc = t == 0 ? term : acc + term;
    }
    out[e] = acc;
}

// element densities of a topology: 1 for solid, the ersatz scale for void
__global__ void k_density(int64_t n, const uint8_t* solid, double void_scale, double* rho) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) rho[e] = solid[e] ? 1.0 : void_scale;
}

__global__ void k_mark(int64_t n, int64_t keep, const int32_t* order, uint8_t* solid, int32_t* order_out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t e = order[i];
    solid[e] = (i < keep) ? 1 : 0;
    if (order_out) order_out[i] = e;
}

}  // namespace

int stress_pnorm(const Grid& g, const double h[3], double E, double nu, const double* rho, const uint8_t* nmask,
                 int nrhs, const double* U, double p, double* vm, double* pn_host, double* B, hipStream_t st) {
    if (nrhs < 1 || nrhs > 4 || !(p >= 2.0) || !std::isfinite(p)) {
        set_error("stress: nrhs 1..4 and p >= 2");
        return AFD_E_INVALID_ARG;
    }
    if (g.nelem >= ((int64_t)1 << 31) || g.nnode >= ((int64_t)1 << 31)) {
        set_error("stress: more than 2^31 elements or nodes");
        return AFD_E_INVALID_ARG;
    }
    StressP P;
    memset(&P, 0, sizeof(P));
    P.nx = g.nx, P.ny = g.ny, P.nz = g.nz;
    P.nrhs = nrhs;
    P.ndof = g.ndof;
    for (int a = 0; a < 3; ++a) P.inv4h[a] = 1.0 / (4.0 * h[a]);
    P.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    P.mu = E / (2.0 * (1.0 + nu));
    P.p = p;
    P.U = U;
    P.rho = rho;
    P.vm = vm;
    const unsigned nb = (unsigned)((g.nelem + 255) / 256);
    double* work = nullptr;
    const size_t part_n = (size_t)nrhs * nb, T_n = B ? (size_t)nrhs * 6 * g.nelem : 0;
    if (afd::dev_malloc((void**)&work, (part_n + T_n) * sizeof(double)) != hipSuccess) {
        set_error("stress: out of device memory");
        return AFD_E_OOM;
    }
    P.part = work;
    P.T = B ? work + part_n : nullptr;
    int rc = AFD_OK;
    std::vector<double> part(part_n);
    hipLaunchKernelGGL(k_stress, dim3(nb, nrhs), dim3(256), 0, st, P);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(part.data(), P.part, part_n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("stress: kernel or copy failed");
        rc = AFD_E_HIP;
    }
    double sum = 0.0;
    for (size_t i = 0; i < part_n; ++i) sum += part[i];
    const double pn = std::pow(sum, 1.0 / p);
    if (rc == AFD_OK && pn_host) *pn_host = pn;
    if (rc == AFD_OK && B) {
        const double scale = sum > 0.0 ? std::pow(pn, 1.0 - p) : 0.0;
        hipLaunchKernelGGL(k_stress_rhs, dim3((unsigned)((g.nnode + 255) / 256), nrhs), dim3(256), 0, st, P, nmask,
                           scale, B);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
            set_error("stress: adjoint right-hand side kernel failed");
            rc = AFD_E_HIP;
        }
    }
    (void)hipStreamSynchronize(st);
    (void)afd::dev_free(work);
    return rc;
}

int launch_combine(int64_t n, int nterms, const double* const* fields, const int* rows, const double* coef,
                   double* out, hipStream_t s) {
    if (nterms < 1 || nterms > MAX_TERMS || n < 1) {
        set_error("combine: 1..4 terms and n >= 1");
        return AFD_E_INVALID_ARG;
    }
    CombineP p;
    memset(&p, 0, sizeof(p));
    p.nterms = nterms;
    for (int t = 0; t < nterms; ++t) {
        if (!fields[t] || rows[t] < 1) {
            set_error("combine: null field or empty group");
            return AFD_E_INVALID_ARG;
        }
        p.f[t] = fields[t];
        p.rows[t] = rows[t];
        p.coef[t] = coef[t];
    }
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, out);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_density(int64_t n, const uint8_t* solid, double void_scale, double* rho, hipStream_t s) {
    hipLaunchKernelGGL(k_density, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, solid, void_scale, rho);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_parting_distance(const int dims[3], int axis, int parting, int32_t* dist, hipStream_t s) {
    const int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
    hipLaunchKernelGGL(k_parting_distance, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dims[0], dims[1],
                       dims[2], axis, parting, dist);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_cast(const int dims[3], int axis, int parting, const double* phi, double* out, hipStream_t s) {
    const int lines = axis == 0 ? dims[1] * dims[2] : (axis == 1 ? dims[0] * dims[2] : dims[0] * dims[1]);
    if (axis == 0)
        hipLaunchKernelGGL(k_cast_x, dim3((lines + 3) / 4), dim3(256), 0, s, dims[0], lines, parting, phi, out);
    else
        hipLaunchKernelGGL(k_cast_yz, dim3((lines + 63) / 64), dim3(256), 0, s, dims[0], dims[1], dims[2], axis,
                           parting, phi, out);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_sensitivity(const Grid& g, const KeHaar& kh, const double* rho, int nfields, const double* const* Ua,
                       const double* const* Ub, double* S, hipStream_t s) {
    if (nfields < 1 || nfields > MAXF) {
        set_error("sensitivity: 1..16 fields");
        return AFD_E_INVALID_ARG;
    }
    if (g.nelem >= ((int64_t)1 << 31) || g.nnode >= ((int64_t)1 << 31)) {
        set_error("sensitivity: more than 2^31 elements or nodes");
        return AFD_E_INVALID_ARG;
    }
    SensP p;
    memset(&p, 0, sizeof(p));
    p.nx = g.nx;
    p.ny = g.ny;
    p.nz = g.nz;
    p.nfields = nfields;
    for (int f = 0; f < nfields; ++f) {
        p.ua[f] = Ua[f];
        p.ub[f] = Ub[f];
    }
    p.kh = kh;
    hipLaunchKernelGGL(k_sensitivity, dim3((unsigned)((g.nelem + 255) / 256)), dim3(256), 0, s, p, rho, S);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

size_t threshold_work_bytes(int64_t n) {
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    // k0, k1 (8 B), i0, i1 (4 B) per key, 256 counters per tile, 256 digit totals;
    // each part rounded to 256 B
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 2 * r((size_t)n * 8) + 2 * r((size_t)n * 4) + r((size_t)256 * ntiles * 4) + r(256 * 4);
}

int threshold_run(const double* s, const int32_t* tie, int64_t n, double vol_frac, uint8_t* solid, int32_t* order,
                  double* tau_host, void* work, hipStream_t st) {
    if (n <= 0 || n > 0x7fffffff || !(vol_frac >= 0.0 && vol_frac <= 1.0)) {
        set_error("threshold: need 0 < n < 2^31 and 0 <= vol_frac <= 1");
        return AFD_E_INVALID_ARG;
    }
    const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char* p = (char*)work;
    uint64_t* k0 = (uint64_t*)p;
    p += r((size_t)n * 8);
    uint64_t* k1 = (uint64_t*)p;
    p += r((size_t)n * 8);
    int32_t* i0 = (int32_t*)p;
    p += r((size_t)n * 4);
    int32_t* i1 = (int32_t*)p;
    p += r((size_t)n * 4);
    uint32_t* hist = (uint32_t*)p;
    p += r((size_t)256 * ntiles * 4);
    uint32_t* dtot = (uint32_t*)p;
    const dim3 eg((unsigned)((n + 255) / 256));
    auto pass = [&](int shift) {
        hipLaunchKernelGGL(k_hist, dim3(ntiles), dim3(RS_T), 0, st, n, k0, shift, hist, ntiles);
        hipLaunchKernelGGL(k_scan_tiles, dim3(256), dim3(256), 0, st, hist, ntiles, dtot);
        hipLaunchKernelGGL(k_scan_digits, dim3(1), dim3(64), 0, st, dtot);
        hipLaunchKernelGGL(k_scatter, dim3(ntiles), dim3(RS_T), 0, st, n, k0, i0, k1, i1, shift, hist, ntiles, dtot);
        std::swap(k0, k1);
        std::swap(i0, i1);
    };
    if (tie) {
        // stable LSD passes: the tie key first, then the 8 bytes of the s key
        hipLaunchKernelGGL(k_make_tie_keys, eg, dim3(256), 0, st, n, tie, k0, i0);
        for (int b = 0; b < 4; ++b) pass(8 * b);
        hipLaunchKernelGGL(k_make_keys_perm, eg, dim3(256), 0, st, n, s, i0, k0);
    } else {
        hipLaunchKernelGGL(k_make_keys, eg, dim3(256), 0, st, n, s, k0, i0);
    }
    for (int b = 0; b < 8; ++b) pass(8 * b);
    int64_t keep = (int64_t)std::ceil(vol_frac * (double)n);
    if (keep > n) keep = n;
    if (keep < 0) keep = 0;
    hipLaunchKernelGGL(k_mark, eg, dim3(256), 0, st, n, keep, i0, solid, order);
    AFD_HIP_TRY(hipGetLastError());
    if (tau_host) {
        *tau_host = INFINITY;
        if (keep > 0) {
            int32_t e = 0;
            AFD_HIP_TRY(hipMemcpyAsync(&e, i0 + keep - 1, 4, hipMemcpyDeviceToHost, st));
            AFD_HIP_TRY(hipStreamSynchronize(st));
            AFD_HIP_TRY(hipMemcpyAsync(tau_host, s + e, 8, hipMemcpyDeviceToHost, st));
        }
    }
    AFD_HIP_TRY(hipStreamSynchronize(st));
    return AFD_OK;
}

// ---- the allocation-free ranking (afd_threshold_noalloc) ----------------
// Its work space is one file-scope device array, `scratch`, sized for
// AFD_THRESHOLD_NOALLOC_MAX keys; every GPU the library runs on holds its own
// copy until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the device
// address of each GPU's copy is taken once per device, with that device
// current, when a context is created on it, and kept here.
static __device__ __align__(256) char scratch[THRESHOLD_NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu;

int threshold_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("threshold scratch: device index beyond 63");
        return AFD_E_NO_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return AFD_OK;
    void* ptr = nullptr;
    AFD_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));  // the current device's copy
    if (!ptr) {
        set_error("threshold scratch: no device address");
        return AFD_E_HIP;
    }
    g_scratch_ptr[device] = ptr;
    return AFD_OK;
}

int threshold_noalloc(int device, const double* s, const int32_t* tie, int64_t n, double vol_frac, uint8_t* solid,
                      int32_t* order, double* tau_host, hipStream_t st) {
    static_assert(THRESHOLD_NOALLOC_BYTES >= 2 * (8 << 21) + 2 * (4 << 21) + 256 * 1024 * 4 + 1024,
                  "scratch smaller than the work space of AFD_THRESHOLD_NOALLOC_MAX keys");
    if (n <= 0 || n > AFD_THRESHOLD_NOALLOC_MAX) {
        set_error("threshold_noalloc: need 0 < n <= AFD_THRESHOLD_NOALLOC_MAX (2097152)");
        return AFD_E_INVALID_ARG;
    }
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (device >= 0 && device < MAX_DEVICES) ptr = g_scratch_ptr[device];
    }
    if (!ptr) {
        set_error("threshold_noalloc: scratch address not set up for this device");
        return AFD_E_HIP;
    }
    if (threshold_work_bytes(n) > THRESHOLD_NOALLOC_BYTES) {
        set_error("threshold_noalloc: work space beyond the scratch array");
        return AFD_E_INVALID_ARG;
    }
    return threshold_run(s, tie, n, vol_frac, solid, order, tau_host, ptr, st);
}

int threshold_gpu(const double* s, const int32_t* tie, int64_t n, double vol_frac, uint8_t* solid, int32_t* order,
                  double* tau_host, hipStream_t st) {
    if (n <= 0 || n > 0x7fffffff) {
        set_error("threshold: need 0 < n < 2^31 and 0 <= vol_frac <= 1");
        return AFD_E_INVALID_ARG;
    }
    void* work = nullptr;
    if (afd::dev_malloc(&work, threshold_work_bytes(n)) != hipSuccess) {
        set_error("threshold: out of device memory");
        return AFD_E_OOM;
    }
    const int rc = threshold_run(s, tie, n, vol_frac, solid, order, tau_host, work, st);
    if (rc != AFD_OK) (void)hipStreamSynchronize(st);  // no kernel may still use the work space
    (void)afd::dev_free(work);
    return rc;
}

}  // namespace afd
