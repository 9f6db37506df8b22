// Operator apply with the dense element contraction on the FP64 matrix cores:
// Y_e = rho_e Ke U_e for all elements of a layer tile, as the batched product
// Ke (24x24, padded to 32 rows) x [U_e1 ... U_e256] (24 x 256) with
// v_mfma_f64_16x16x4f64, one launch for all right-hand sides (blockIdx.y).
//
// Same traversal as the VALU kernel (16x16 element tile per workgroup, z
// marching, overlapped tiles owning 15x15 nodes, fixed-order gather); only the
// element step differs.  Wave w of a workgroup owns element rows 4w..4w+3:
// one 16-column MFMA tile per row.
#include "afd_internal.h"

namespace afd {

namespace {

constexpr int TX = 16, TY = 16, NT = TX * TY;
constexpr int PX = TX + 1, PY = TY + 1;
constexpr int PLANE = PX * PY * 3;
constexpr int SPT = (PLANE + NT - 1) / NT;

typedef double d4 __attribute__((ext_vector_type(4)));

struct MfP {
    int nx, ny, nz;
    int tiles_x, tiles_y, zc, nchunk;
    int64_t ndof;
    const double* rho;
    const uint8_t* nmask;
    const double* U;
    double* Y;
    const double* ke;  // 24x24 row-major, LOCAL node order
};

// DOF index in LOCAL order (3a + c) of DOF (bit-pattern corner n, component c)
__device__ __forceinline__ int local_of_bit(int n) {
    // bit pattern ax + 2 ay + 4 az -> LOCAL index (bottom face CCW, then top)
    const int ax = n & 1, ay = (n >> 1) & 1, az = n >> 2;
    const int face = ay ? (ax ? 2 : 3) : (ax ? 1 : 0);
    return face + 4 * az;
}

__global__ __launch_bounds__(NT) void k_matvec_mfma(MfP P) {
    __shared__ double plane[2][PLANE];
    __shared__ double outb[24][NT];
    __shared__ double rl[NT];

    const int rhs = blockIdx.y;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lx = t % TX, ly = t / TX;
    const int tile = blockIdx.x % (P.tiles_x * P.tiles_y);
    const int chunk = blockIdx.x / (P.tiles_x * P.tiles_y);
    const int X0 = (tile % P.tiles_x) * (TX - 1) - 1;
    const int Y0 = (tile / P.tiles_x) * (TY - 1) - 1;
    const int Z0 = chunk * P.zc;
    const int Z1 = min(Z0 + P.zc, P.nz + 1);
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int64_t sy = nx + 1, sz = (int64_t)(nx + 1) * (ny + 1);
    const double* U = P.U + (int64_t)rhs * P.ndof;
    double* Y = P.Y + (int64_t)rhs * P.ndof;
    const int gi = X0 + lx, gj = Y0 + ly;
    const bool own = lx >= 1 && ly >= 1 && gi <= nx && gj <= ny;
    const bool elem_xy = gi >= 0 && gi < nx && gj >= 0 && gj < ny;

    // A operand (Ke rows in corner-bit order), 2 row tiles x 6 k-steps:
    // lane holds row 16*mt + lane%16, column 4*s + lane/16
    double Aop[2][6];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const int row = 16 * mt + (lane & 15), col = 4 * s + (lane >> 4);
            double v = 0.0;
            if (row < 24) {
                const int lr = 3 * local_of_bit(row / 3) + row % 3;
                const int lc = 3 * local_of_bit(col / 3) + col % 3;
                v = P.ke[lr * 24 + lc];
            }
            Aop[mt][s] = v;
        }
    // B operand sources: for k-step s this lane reads DOF k = 4s + lane/16 of
    // element (lane%16, row); corner bit nb = k/3, comp c = k%3
    int boff[6], bpl[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int k = 4 * s + (lane >> 4);
        const int nb = k / 3, c = k % 3;
        boff[s] = (((nb >> 1) & 1) * PX + (lane & 15) + (nb & 1)) * 3 + c;  // + row*PX*3 later
        bpl[s] = nb >> 2;
    }

    int64_t soff[SPT];
    int sc_[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int f = t + q * NT;
        soff[q] = -1;
        sc_[q] = 0;
        if (f < PLANE) {
            const int row = f / (PX * 3);
            const int rem = f - row * (PX * 3);
            const int li = rem / 3;
            const int i = X0 + li, j = Y0 + row;
            sc_[q] = rem - li * 3;
            if (i >= 0 && i <= nx && j >= 0 && j <= ny) soff[q] = i + sy * j;
        }
    }
    auto fetch = [&](int gk, double reg[SPT]) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            double v = 0.0;
            if (soff[q] >= 0 && gk >= 0 && gk <= nz) {
                const int64_t node = soff[q] + sz * gk;
                if (!((P.nmask[node] >> sc_[q]) & 1)) v = U[3 * node + sc_[q]];
            }
            reg[q] = v;
        }
    };
    auto put = [&](int buf, const double reg[SPT]) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int f = t + q * NT;
            if (f < PLANE) plane[buf][f] = reg[q];
        }
    };
    auto rho_at = [&](int k) -> double {
        return (elem_xy && k >= 0 && k < nz) ? P.rho[gi + (int64_t)nx * (gj + (int64_t)ny * k)] : 0.0;
    };

    double carry[3] = {0.0, 0.0, 0.0};
    double reg[SPT];
    fetch(Z0 - 1, reg);
    put(0, reg);
    fetch(Z0, reg);
    put(1, reg);
    double rho_cur = rho_at(Z0 - 1);
    int buf = 1;  // holds plane k+1; buf^1 holds plane k

    for (int k = Z0 - 1; k < Z1; ++k) {
        const bool more = k + 2 <= Z1;
        if (more) fetch(k + 2, reg);
        const double rho_nxt = rho_at(k + 1);
        rl[t] = rho_cur;
        __syncthreads();  // planes k, k+1 and densities staged
        // four 16-element column tiles per wave (element rows 4w..4w+3)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 4 * w + q;
            d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const double b = plane[bpl[s] ? buf : (buf ^ 1)][boff[s] + row * PX * 3];
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Aop[0][s], b, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Aop[1][s], b, acc1, 0, 0, 0);
            }
            // D layout: lane holds rows lane/16 + 4v (v = 0..3) of column lane%16
            const int e = row * TX + (lane & 15);
            const double r = rl[e];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r0 = (lane >> 4) + 4 * v;
                outb[r0][e] = r * acc0[v];
                if (16 + r0 < 24) outb[16 + r0][e] = r * acc1[v];
            }
        }
        __syncthreads();
        if (own) {
            const int t00 = t - TX - 1, t10 = t - TX, t01 = t - 1, t11 = t;
            double bot[3], top[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bot[c] = outb[3 * 3 + c][t00] + outb[2 * 3 + c][t10] + outb[1 * 3 + c][t01] + outb[0 * 3 + c][t11];
                top[c] = outb[7 * 3 + c][t00] + outb[6 * 3 + c][t10] + outb[5 * 3 + c][t01] + outb[4 * 3 + c][t11];
            }
            if (k >= Z0) {
                const int64_t node = gi + sy * gj + sz * k;
                const uint8_t m = P.nmask[node];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t a = 3 * node + c;
                    Y[a] = ((m >> c) & 1) ? U[a] : carry[c] + bot[c];
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) carry[c] = top[c];
        }
        __syncthreads();  // planes and outputs consumed before restaging
        if (more) put(buf ^ 1, reg);
        buf ^= 1;
        rho_cur = rho_nxt;
    }
}

}  // namespace

int launch_apply_mfma(const MatvecArgs& a, const double* ke576, int nrhs, const double* U, double* Y,
                      hipStream_t s) {
    if (nrhs < 1 || nrhs > 4) {
        set_error("nrhs must be in 1..4");
        return AFD_E_INVALID_ARG;
    }
    MfP p{};
    p.nx = a.g.nx;
    p.ny = a.g.ny;
    p.nz = a.g.nz;
    p.tiles_x = (a.g.nx + 1 + (TX - 2)) / (TX - 1);
    p.tiles_y = (a.g.ny + 1 + (TY - 2)) / (TY - 1);
    const int planes = a.g.nz + 1;
    int want = (1024 + p.tiles_x * p.tiles_y - 1) / (p.tiles_x * p.tiles_y);
    p.zc = (planes + want - 1) / want;
    if (p.zc < 8) p.zc = 8;
    if (p.zc > planes) p.zc = planes;
    p.nchunk = (planes + p.zc - 1) / p.zc;
    p.ndof = a.g.ndof;
    p.rho = a.rho;
    p.nmask = a.nmask;
    p.U = U;
    p.Y = Y;
    p.ke = ke576;
    dim3 grid(p.tiles_x * p.tiles_y * p.nchunk, nrhs);
    hipLaunchKernelGGL(k_matvec_mfma, grid, dim3(NT), 0, s, p);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

}  // namespace afd
