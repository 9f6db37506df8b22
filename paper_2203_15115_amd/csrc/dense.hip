// Coarse problem of the deflated CG (Sec. 3.5): E = W^T A W for W holding the
// six rigid-body motions of every agglomerated block, its Cholesky factor,
// and the solve mu = E^-1 g used once per iteration.
//
// Ordering: blocks are numbered with the two axes of fewest blocks fastest, so
// E (27-neighbour 6x6 block stencil) has half bandwidth
// w = 6 (n0 n1 + n0 + 1) + 5.  Cutting the ordered unknowns into super-blocks
// of P >= w makes E block tridiagonal: diagonal blocks D_k, sub-diagonal blocks
// B_k = E_{k+1,k}.  The block Cholesky E = L L^T gives
//   L_kk L_kk^T = D_k - C_{k-1} C_{k-1}^T,   C_k = L_{k+1,k} = B_k L_kk^-T,
// and the solve is then a chain of dense matrix-vector products with
// precomputed matrices (no triangular solve on the critical path):
//   forward  x_k = Linv_k g_k - T_k x_{k-1},        T_k = Linv_k C_{k-1}
//   backward mu_k = Linv_k^T x_k - U_k mu_{k+1},    U_k = Linv_k^T C_k^T.
// A pivot that falls below 1e-10 of the original diagonal marks a
// rank-deficient coarse column (e.g. a block whose nodes are all fixed); it
// is dropped: its row and column of Linv are zeroed, so its mu is 0.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "afd_internal.h"

namespace afd {

namespace {

constexpr int NB = 64;  // tile of the blocked dense kernels
constexpr double DROP_TOL = 1e-10;

// ------------------------------------------------------------------ GEMM
// C[M x N] = alpha * op(A) op(B) + beta * C, row-major, FP64.
// op(A)(i,k) = ta ? A[k*lda + i] : A[i*lda + k]; op(B)(k,j) = tb ? B[j*ldb + k] : B[k*ldb + j]
constexpr int GT = 64, GK = 16;
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, double alpha, const double* A, int lda, int ta,
                                              const double* B, int ldb, int tb, double beta, double* C, int ldc) {
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int t = threadIdx.x;
    const int tr = t / 16, tc = t % 16;  // 16x16 threads, 4x4 outputs each
    const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += GK) {
        for (int e = t; e < GT * GK; e += 256) {
            // A tile: rows i0..i0+63, cols k0..k0+15
            int ii, kk;
            if (ta) {
                ii = e % GT;
                kk = e / GT;
            } else {
                kk = e % GK;
                ii = e / GK;
            }
            const int gi = i0 + ii, gk = k0 + kk;
            double av = 0.0;
            if (gi < M && gk < K) av = ta ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
            As[kk][ii] = av;
            int jj, kb;
            if (tb) {
                kb = e % GK;
                jj = e / GK;
            } else {
                jj = e % GT;
                kb = e / GT;
            }
            const int gj = j0 + jj, gkb = k0 + kb;
            double bv = 0.0;
            if (gj < N && gkb < K) bv = tb ? B[(int64_t)gj * ldb + gkb] : B[(int64_t)gkb * ldb + gj];
            Bs[kb][jj] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[kk][tr + 16 * q];
                b[q] = Bs[kk][tc + 16 * q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[q][u] = fma(a[q], b[u], acc[q][u]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int gi = i0 + tr + 16 * q, gj = j0 + tc + 16 * u;
            if (gi < M && gj < N) {
                double* c = C + (int64_t)gi * ldc + gj;
                *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * acc[q][u];
            }
        }
}

// The same product on the FP64 matrix cores: a 64 x 64 tile of C per
// workgroup, 2 x 2 wavefronts of 32 x 32, each a 2 x 2 set of
// v_mfma_f64_16x16x4f64 tiles; K in steps of 16 staged through LDS, the next
// step's operands prefetched into registers while the current one is
// multiplied.  Operand layouts of the instruction (64 lanes): A lane l holds
// (row l % 16, k l / 16), B lane l holds (k l / 16, col l % 16), and
// accumulator register v of lane l is (row l / 16 + 4 v, col l % 16).
typedef double dacc4 __attribute__((ext_vector_type(4)));
// Split K: workgroup z of gridDim.z covers k in [z kchunk, (z + 1) kchunk) and
// writes its partial product to C + z czs (beta must then be 0).
__global__ __launch_bounds__(256) void k_gemm_mfma(int M, int N, int K, double alpha, const double* A, int lda,
                                                   int ta, const double* B, int ldb, int tb, double beta, double* C,
                                                   int ldc, int kchunk, int64_t czs, int64_t azs = 0, int64_t bzs = 0,
                                                   int batched = 0) {
    __shared__ double As[GK][GT + 2];
    __shared__ double Bs[GK][GT + 2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = wv >> 1, wc = wv & 1;
    const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
    // blockIdx.z: a slice of K (partial products at C + z czs), or with
    // batched a separate product A + z azs, B + z bzs -> C + z czs
    const int kbeg = batched ? 0 : blockIdx.z * kchunk, kend = batched ? K : min(K, kbeg + kchunk);
    C += blockIdx.z * czs;
    if (batched) {
        A += blockIdx.z * azs;
        B += blockIdx.z * bzs;
    }
    // loader: element e = t + 256 q (q < 4) of the 64 x 16 A tile and the 16 x 64 B tile
    double ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            int ii, kk;
            if (ta) { ii = e % GT; kk = e / GT; } else { kk = e % GK; ii = e / GK; }
            const int gi = i0 + ii, gk = k0 + kk;
            ra[q] = (gi < M && gk < kend) ? (ta ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk]) : 0.0;
            int jj, kb;
            if (tb) { kb = e % GK; jj = e / GK; } else { jj = e % GT; kb = e / GT; }
            const int gj = j0 + jj, gkb = k0 + kb;
            rb[q] = (gj < N && gkb < kend) ? (tb ? B[(int64_t)gj * ldb + gkb] : B[(int64_t)gkb * ldb + gj]) : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            int ii, kk;
            if (ta) { ii = e % GT; kk = e / GT; } else { kk = e % GK; ii = e / GK; }
            As[kk][ii] = ra[q];
            int jj, kb;
            if (tb) { kb = e % GK; jj = e / GK; } else { jj = e % GT; kb = e / GT; }
            Bs[kb][jj] = rb[q];
        }
    };
    dacc4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dacc4{0.0, 0.0, 0.0, 0.0};
    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        __syncthreads();  // previous step's operands consumed
        store();
        __syncthreads();
        if (k0 + GK < kend) load(k0 + GK);
#pragma unroll
        for (int sk = 0; sk < GK / 4; ++sk) {
            const int kk = 4 * sk + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[kk][32 * wr + 16 * a + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kk][32 * wc + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = i0 + 32 * wr + 16 * a + (lane >> 4) + 4 * v;
                const int gj = j0 + 32 * wc + 16 * b + (lane & 15);
                if (gi < M && gj < N) {
                    double* c = C + (int64_t)gi * ldc + gj;
                    *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * acc[a][b][v];
                }
            }
}

int gemm(int M, int N, int K, double alpha, const double* A, int lda, int ta, const double* B, int ldb, int tb,
         double beta, double* C, int ldc, hipStream_t s) {
    if (M <= 0 || N <= 0) return AFD_OK;
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
    if (K <= 0) {
        hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc);
    } else {
        hipLaunchKernelGGL(k_gemm_mfma, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc,
                           K, (int64_t)0);
    }
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

// dst[i][j] = sum_z src[z][i][j] (M x N, row strides ld / ldd, batch stride zs)
__global__ void k_sum_split(int M, int N, int S, const double* src, int ld, int64_t zs, double* dst, int ldd) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= N) return;
    double v = 0.0;
    for (int z = 0; z < S; ++z) v += src[z * zs + (int64_t)i * ld + j];
    dst[(int64_t)i * ldd + j] = v;
}

// nbatch products C_z = alpha A_z B_z + beta C_z (no transposes), X_z = X + z xzs
int gemm_batched(int nbatch, int M, int N, int K, double alpha, const double* A, int lda, int64_t azs,
                 const double* B, int ldb, int64_t bzs, double beta, double* C, int ldc, int64_t czs, hipStream_t s) {
    if (nbatch <= 0 || M <= 0 || N <= 0 || K <= 0) return AFD_OK;
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, nbatch);
    hipLaunchKernelGGL(k_gemm_mfma, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, K, czs,
                       azs, bzs, 1);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

// C = alpha op(A) op(B) with K split over S workgroup slices whose partial
// products go to part (S x M x ldp) and are then summed into C: for the
// short-and-wide products whose output tiles alone cannot fill the GPU
int gemm_split(int M, int N, int K, double alpha, const double* A, int lda, int ta, const double* B, int ldb, int tb,
               double* C, int ldc, double* part, int ldp, int S, hipStream_t s) {
    if (M <= 0 || N <= 0) return AFD_OK;
    const int kchunk = ((K + S - 1) / S + GK - 1) / GK * GK;
    S = (K + kchunk - 1) / kchunk;
    if (S <= 1) return gemm(M, N, K, alpha, A, lda, ta, B, ldb, tb, 0.0, C, ldc, s);
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, S);
    const int64_t zs = (int64_t)M * ldp;
    hipLaunchKernelGGL(k_gemm_mfma, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, ta, B, ldb, tb, 0.0, part, ldp,
                       kchunk, zs);
    hipLaunchKernelGGL(k_sum_split, dim3((N + 255) / 256, M), dim3(256), 0, s, M, N, S, (const double*)part, ldp, zs,
                       C, ldc);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

// ---------------------------------------------------------- dense Cholesky
// 1/sqrt(d) for a positive normal d: the hardware estimate refined by three
// Newton steps y <- y + y (1 - d y^2) / 2, each of which roughly doubles the
// number of correct bits (full precision to within about one unit in the
// last place from an estimate good to 12 bits)
__device__ __forceinline__ double rsqrt_newton(double d) {
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        const double e = fma(-d * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// Factor the nb x nb diagonal tile at (j0, j0) of the row-major P x P matrix
// A in place (lower), with dropping; write the tile inverse (rows/cols of
// dropped pivots zeroed) to the same position of Linv.
__global__ __launch_bounds__(256) void k_potrf_tile(double* A, double* Linv, int P, int j0, int nb,
                                                    const double* ediag, int32_t* dropped) {
    static_assert(NB == 64, "the register layout assumes 64 x 64 tiles and 256 threads");
    // Right-looking Cholesky of the tile and, alongside, the forward
    // substitution L X = I, written to be nearly free of divergent branches
    // (the tile factorisation is a chain of 64 dependent steps; branches and
    // barriers set its pace).  Thread (r, q0) owns row r of L and of X at
    // columns q0 + 4 i.  The pivot loop is rolled over 16 groups of 4
    // (unrolled) pivots; within group g the L registers are shifted so that
    // column q0 + 4 (g + i) sits in Lr[i].  Each step reads the not yet
    // scaled column c of L and row c of X from LDS (double buffered,
    // published at the end of the previous step: one barrier per pivot):
    //  * rows above the pivot get a zero row factor, so their updates are
    //    no-ops; only Lr[0] needs a mask (its column may be <= c);
    //  * the column buffer is padded with zeros to 2 NB entries and the X row
    //    is zero beyond column c, so the updates read fixed offsets;
    //  * entries above the diagonal of L take garbage updates but are never
    //    published or stored;
    //  * threads that do not own the published column store to a slot of
    //    their own.
    __shared__ double ucol[2][2 * NB];  // column c of the partly factored tile, rows >= c, not scaled
    __shared__ double urow[2][NB];      // row c of X, not scaled (zero beyond column c)
    __shared__ double dummy[256];
    __shared__ double ed[NB];           // diagonal of E (drop test)
    __shared__ int drop[NB];
    const int t = threadIdx.x;
    const int r = t >> 2, q0 = t & 3;
    for (int i = t; i < 2 * 2 * NB; i += 256) (&ucol[0][0])[i] = 0.0;
    for (int i = t; i < 2 * NB; i += 256) (&urow[0][0])[i] = 0.0;
    __syncthreads();
    double Lr[16], Xr[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = q0 + 4 * i;
        // rows beyond nb are padded with the identity (pivot 1, never dropped)
        Lr[i] = (r < nb && q <= r) ? A[(int64_t)(j0 + r) * P + j0 + q] : (r == q ? 1.0 : 0.0);
        Xr[i] = (r == q) ? 1.0 : 0.0;
    }
    if (t < NB) ed[t] = t < nb ? ediag[j0 + t] : 1.0;
    if (q0 == 0) ucol[0][r] = Lr[0];
    if (t == 0) urow[0][0] = 1.0;
    for (int g = 0; g < NB / 4; ++g) {
        const int cb = q0 + 4 * g;  // column of Lr[0]
#pragma unroll
        for (int qc = 0; qc < 4; ++qc) {
            const int c = 4 * g + qc, b = qc & 1;
            __syncthreads();
            const double d = ucol[b][c];
            const double edc = ed[c];
            const bool dr = !(edc > 0.0) || !(d > DROP_TOL * edc);
            // 1/sqrt(d) once; 1/d and sqrt(d) follow from it by one product each
            // (the estimate needs a normal argument well inside the range; a
            // pivot as small as 2^-900 only arises for E near the denormals)
            const double pi = dr ? 1.0 : (d > 0x1p-900 ? rsqrt_newton(d) : 1.0 / sqrt(d));
            const double id = dr ? 0.0 : pi * pi;
            const double f = r > c ? ucol[b][r] * id : 0.0;
            const double* uc = &ucol[b][cb];
            const double* ur = &urow[b][q0];
            Lr[0] = fma(q0 > qc ? -f : 0.0, uc[0], Lr[0]);
#pragma unroll
            for (int i = 1; i < 16; ++i) Lr[i] = fma(-f, uc[4 * i], Lr[i]);
#pragma unroll
            for (int i = 0; i < 16; ++i) Xr[i] = fma(-f, ur[4 * i], Xr[i]);
            // publish column c + 1 and row c + 1 of X for the next step
            if (c + 1 < NB) {
                const bool own = q0 == ((qc + 1) & 3) && r > c;
                *(own ? &ucol[b ^ 1][r] : &dummy[t]) = qc == 3 ? Lr[1] : Lr[0];
                if (r == c + 1) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) urow[b ^ 1][q0 + 4 * i] = Xr[i];
                }
            }
            // column c of L and row c of X are final once scaled
            const double pv = dr ? 1.0 : d * pi;
            if (q0 == qc) Lr[0] = r > c ? (dr ? 0.0 : Lr[0] * pi) : (r == c ? pv : Lr[0]);
            if (r == c) {
#pragma unroll
                for (int i = 0; i < 16; ++i) Xr[i] *= pi;
            }
            drop[c] = dr ? 1 : 0;  // every thread stores the same value
        }
        // column cb of L is final: store it and shift the rest down
        if (r < nb && cb <= r) A[(int64_t)(j0 + r) * P + j0 + cb] = Lr[0];
#pragma unroll
        for (int i = 0; i < 15; ++i) Lr[i] = Lr[i + 1];
        Lr[15] = 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = q0 + 4 * i;
        if (r < nb && q <= r) Linv[(int64_t)(j0 + r) * P + j0 + q] = (drop[r] || drop[q]) ? 0.0 : Xr[i];
    }
    if (t < nb) dropped[j0 + t] = drop[t];
}

// panel rows r >= j0+nb, cols j0..j0+nb-1:  A_rc <- sum_t A_rt Tinv_ct  (Tinv = diag tile of Linv)
__global__ __launch_bounds__(256) void k_panel(double* A, const double* Linv, int P, int j0, int nb) {
    __shared__ double Ti[NB][NB + 1];
    __shared__ double Ar[64][NB + 1];
    const int t = threadIdx.x;
    const int r = t >> 2, q0 = t & 3;  // thread owns panel row r, columns q0 + 4 i
    const int r0 = j0 + nb + blockIdx.x * 64;
    const int gr = r0 + r;
#pragma unroll 4
    for (int i = 0; i < NB / 4; ++i) {
        const int q = q0 + 4 * i;
        Ti[r][q] = (r < nb && q < nb) ? Linv[(int64_t)(j0 + r) * P + j0 + q] : 0.0;
        Ar[r][q] = (gr < P && q < nb) ? A[(int64_t)gr * P + j0 + q] : 0.0;
    }
    __syncthreads();
    if (gr >= P) return;
    double acc[NB / 4];
#pragma unroll
    for (int i = 0; i < NB / 4; ++i) acc[i] = 0.0;
    for (int q = 0; q < nb; ++q) {
        const double a = Ar[r][q];
#pragma unroll
        for (int i = 0; i < NB / 4; ++i) acc[i] = fma(a, Ti[q0 + 4 * i][q], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < NB / 4; ++i) {
        const int c = q0 + 4 * i;
        if (c < nb) A[(int64_t)gr * P + j0 + c] = acc[i];
    }
}

__global__ void k_zero_dropped(double* Linv, int P, const int32_t* dropped) {
    const int r = blockIdx.y;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P; c += gridDim.x * blockDim.x)
        if (dropped[r] || dropped[c]) Linv[(int64_t)r * P + c] = 0.0;
}

__global__ void k_transpose(int P, const double* A, double* B) {
    __shared__ double tile[32][33];
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    for (int q = threadIdx.y; q < 32; q += blockDim.y) {
        const int r = y0 + q, c = x0 + threadIdx.x;
        if (r < P && c < P) tile[q][threadIdx.x] = A[(int64_t)r * P + c];
    }
    __syncthreads();
    for (int q = threadIdx.y; q < 32; q += blockDim.y) {
        const int r = x0 + q, c = y0 + threadIdx.x;
        if (r < P && c < P) B[(int64_t)r * P + c] = tile[threadIdx.x][q];
    }
}

// -------------------------------------------------------------- assembly
// Where entry (row, col) of E lives in the two-ended order (positions kr, kc of
// row and column): the diagonal super-block D[kr], the coupling B[kc] to the
// next position, or, for the middle (position K-1) against the end of chain A
// (position m-1), B[m-1] (that slot couples nothing else: chain A's end and
// chain B's start are not neighbours).  Entries above the diagonal are not
// stored.  Returns null for them.
__host__ __device__ inline double* coarse_slot(double* D, double* B, int P, int K, int m, int row, int col) {
    const int kr = row / P, kc = col / P;
    const int64_t at = (int64_t)(row % P) * P + col % P;
    if (kr == kc) return D + (int64_t)kr * P * P + at;
    // (positions m and m-1 are not neighbours: B[m-1] holds the middle's coupling)
    if ((kr == kc + 1 && kc != m - 1) || (kr == K - 1 && kc == m - 1)) return B + (int64_t)kc * P * P + at;
    return nullptr;
}

struct ScatP {
    int nb[3];
    int P, ncoarse, K, m;
    const int32_t* perm;  // natural coarse index -> position
};

// one thread per (block J, row mode m'): E[(J,m'),(I,m)] = G[6J+m'] with I the
// block of `color` adjacent to J
__global__ void k_scatter_probe(ScatP p, const double* G, int color, int mode, double* D, double* B) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int nblk = p.nb[0] * p.nb[1] * p.nb[2];
    if (q >= 6 * nblk) return;
    const int J = q / 6, mr = q % 6;
    const int jb[3] = {J % p.nb[0], (J / p.nb[0]) % p.nb[1], J / (p.nb[0] * p.nb[1])};
    const int cc[3] = {color % 3, (color / 3) % 3, color / 9};
    int ib[3];
    for (int a = 0; a < 3; ++a) {
        ib[a] = -1;
        for (int d = -1; d <= 1; ++d) {
            const int v = jb[a] + d;
            if (v >= 0 && v < p.nb[a] && v % 3 == cc[a]) ib[a] = v;
        }
        if (ib[a] < 0) return;
    }
    const int I = ib[0] + p.nb[0] * (ib[1] + p.nb[1] * ib[2]);
    double* at = coarse_slot(D, B, p.P, p.K, p.m, p.perm[6 * J + mr], p.perm[6 * I + mode]);
    if (at) *at = G[6 * J + mr];
}

// E = W^T A W formed directly from the element matrices.  The six motions are
// written in grid-index coordinates; with equal voxel edges they are rigid, so
// A w vanishes inside a block and only elements with nodes in two or more
// blocks (or with fixed DOFs, where W is cut) contribute.  With unequal edges
// the index-space rotations strain the voxels and every element touching the
// block is taken.  One workgroup per block I
// walks, in a fixed order, the elements touching I's nodes; for each it forms
// rho_e Ke u_a for the six modes u_a of I (zero at other blocks' nodes and at
// fixed DOFs) and every thread adds, for its own entries (a, J, b), the
// products with mode b of block J over the element's nodes in J.  Each entry
// has one owner and a fixed summation order: deterministic.
struct DirP {
    int n[3];          // elements per axis
    int b[3], nb[3];   // block edge (elements) and blocks per axis
    double inv_scale;
    int P, ncoarse, K, m;
    const int32_t* perm;
    const double* rho;  // per element
    const uint8_t* nm;  // per node: bit c set when DOF c is fixed
    const double* ke;   // 24 x 24, row-major, local node order
    int rigid;          // 1: the motions are strain-free (equal voxel edges)
};

__device__ __forceinline__ double block_centre(const DirP& p, int ax, int bb) {
    const int lo = bb * p.b[ax], hi = (bb == p.nb[ax] - 1) ? p.n[ax] : lo + p.b[ax] - 1;
    return 0.5 * (lo + hi);
}
// component c of rigid mode m of the block with centre cc at node (i, j, k)
// (translations m = 0..2 along axis m; rotations m = 3..5 about axis r = m - 3:
// component r + 1 is -x[r + 2], component r + 2 is +x[r + 1], indices mod 3)
__device__ __forceinline__ double rigid_mode(const DirP& p, int m, int c, const int nd[3], const double cc[3]) {
    const double x[3] = {(nd[0] - cc[0]) * p.inv_scale, (nd[1] - cc[1]) * p.inv_scale, (nd[2] - cc[2]) * p.inv_scale};
    const int r = m - 3, c1 = r == 2 ? 0 : r + 1, c2 = r == 0 ? 2 : r - 1;  // r + 1, r + 2 (mod 3)
    const double rot = c == c1 ? -x[c2] : (c == c2 ? x[c1] : 0.0);
    return m < 3 ? (m == c ? 1.0 : 0.0) : rot;
}

// STAGE: the densities and fixity of the element box are first copied to LDS
// (dynamic shared memory: densities, then fixity bytes), so the element walk
// waits on no global load; taken when the largest box fits.
template <bool STAGE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_coarse_direct(DirP p, double* D, double* B) {
    extern __shared__ double box[];
    __shared__ double uI[6][24];     // modes of I on the element (zero off I and at fixed DOFs)
    __shared__ double vJ[6][24];     // modes of each node's own block (zero at fixed DOFs)
    __shared__ double f[6][24];      // rho_e Ke uI
    __shared__ double Mk[8][36];     // node k's share: sum_c f[a][3k+c] vJ[b][3k+c], at [k][6a+b]
    const int t = threadIdx.x;
    // workgroups go round-robin over the 8 XCDs: give each XCD a contiguous
    // range of blocks, so neighbours (overlapping element boxes) share an L2
    const int I = (blockIdx.x % 8) * (gridDim.x / 8) + min((int)(blockIdx.x % 8), (int)(gridDim.x % 8)) +
                  (int)(blockIdx.x / 8);
    const int ib[3] = {I % p.nb[0], (I / p.nb[0]) % p.nb[1], I / (p.nb[0] * p.nb[1])};
    double ci[3];
    int e0[3], e1[3], lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        ci[a] = block_centre(p, a, ib[a]);
        lo[a] = ib[a] * p.b[a];
        hi[a] = (ib[a] == p.nb[a] - 1) ? p.n[a] : lo[a] + p.b[a] - 1;
        e0[a] = max(lo[a] - 1, 0);
        e1[a] = min(hi[a], p.n[a] - 1);
    }
    const int EX = e1[0] - e0[0] + 1, EY = e1[1] - e0[1] + 1, EZ = e1[2] - e0[2] + 1;
    const int nel = EX * EY * EZ;
    uint8_t* nmb = reinterpret_cast<uint8_t*>(box + nel);
    if (STAGE) {
        for (int i = t; i < nel; i += 256) {
            const int lx = i % EX, ly = (i / EX) % EY, lz = i / (EX * EY);
            box[i] = p.rho[(e0[0] + lx) + p.n[0] * ((e0[1] + ly) + p.n[1] * (e0[2] + lz))];
        }
        const int nnb = (EX + 1) * (EY + 1) * (EZ + 1);
        for (int i = t; i < nnb; i += 256) {
            const int lx = i % (EX + 1), ly = (i / (EX + 1)) % (EY + 1), lz = i / ((EX + 1) * (EY + 1));
            nmb[i] = p.nm[(e0[0] + lx) + (p.n[0] + 1) * ((e0[1] + ly) + (p.n[1] + 1) * (e0[2] + lz))];
        }
    }
    // this thread's slot of the element vectors: mode m, DOF d = 3 n + c, and
    // column d of Ke (= row d: Ke is symmetric) held in registers
    const int m = t / 24, d = t % 24, n = d / 3, c = d % 3;
    double kc[24];
#pragma unroll
    for (int dd = 0; dd < 24; ++dd) kc[dd] = t < 144 ? p.ke[dd * 24 + d] : 0.0;
    // owned entries: pair ab = 6 a + b = t % 36 (mode a of I, mode b of J) for
    // the neighbours J = I + (dx, dy, dz) of code jr = t / 36 + 7 s (threads < 252)
    const int ab = t % 36, jr0 = t / 36;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int sy = p.n[0] + 1, sz = (p.n[0] + 1) * (p.n[1] + 1);
    __syncthreads();
    // a node's block offset along an axis: -1, 0 or 1 (digit 0, 1, 2)
    auto digit = [](int i, int l, int h) { return i < l ? 0 : (i > h ? 2 : 1); };
    for (int ez = e0[2]; ez <= e1[2]; ++ez)
    for (int ey = e0[1]; ey <= e1[1]; ++ey)
    for (int ex = e0[0]; ex <= e1[0]; ++ex) {
        // the element's nodes (public local order): block offset code and fixity
        const int gx[2] = {digit(ex, lo[0], hi[0]), digit(ex + 1, lo[0], hi[0])};
        const int gy[2] = {digit(ey, lo[1], hi[1]), digit(ey + 1, lo[1], hi[1])};
        const int gz[2] = {digit(ez, lo[2], hi[2]), digit(ez + 1, lo[2], hi[2])};
        int rel[8];
        uint8_t fx[8];
        bool interior = true;
        // first node's fixity index and the strides to the others
        const int f0 = STAGE ? (ex - e0[0]) + (EX + 1) * ((ey - e0[1]) + (EY + 1) * (ez - e0[2]))
                             : ex + sy * (ey + (p.n[1] + 1) * ez);
        const int fy = STAGE ? EX + 1 : sy, fz = STAGE ? (EX + 1) * (EY + 1) : sz;
        const uint8_t* fb = STAGE ? nmb : p.nm;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int bx = ((a + 1) >> 1) & 1, by = (a >> 1) & 1, bz = a >> 2;
            rel[a] = gx[bx] + 3 * gy[by] + 9 * gz[bz];  // 13: block I itself
            fx[a] = fb[f0 + bx + by * fy + bz * fz];
            interior = interior & (rel[a] == 13) & (fx[a] == 0);  // no short circuit: the reads issue together
        }
        if (interior && p.rigid) continue;  // every thread takes the same branch
        if (t < 144) {
            const int nd[3] = {ex + (((n + 1) >> 1) & 1), ey + ((n >> 1) & 1), ez + (n >> 2)};
            const int r = rel[n];
            const bool free_dof = !((fx[n] >> c) & 1);
            const double cj[3] = {block_centre(p, 0, ib[0] + r % 3 - 1), block_centre(p, 1, ib[1] + (r / 3) % 3 - 1),
                                  block_centre(p, 2, ib[2] + r / 9 - 1)};
            uI[m][d] = (free_dof && r == 13) ? rigid_mode(p, m, c, nd, ci) : 0.0;
            vJ[m][d] = free_dof ? rigid_mode(p, m, c, nd, cj) : 0.0;
        }
        __syncthreads();
        if (t < 144) {  // Ke is symmetric: read its column d (consecutive across lanes)
            double s4v[4] = {0.0, 0.0, 0.0, 0.0};  // four partial sums: a short dependent chain
#pragma unroll
            for (int dd = 0; dd < 24; ++dd) s4v[dd & 3] = fma(kc[dd], uI[m][dd], s4v[dd & 3]);
            f[m][d] = (STAGE ? box[(ex - e0[0]) + EX * ((ey - e0[1]) + EY * (ez - e0[2]))]
                             : p.rho[ex + p.n[0] * (ey + p.n[1] * ez)]) *
                      ((s4v[0] + s4v[1]) + (s4v[2] + s4v[3]));
        }
        __syncthreads();
        for (int e = t; e < 288; e += 256) {
            const int k = e / 36, a = (e % 36) / 6, b = e % 6;
            double v = f[a][3 * k] * vJ[b][3 * k];
            v = fma(f[a][3 * k + 1], vJ[b][3 * k + 1], v);
            Mk[k][6 * a + b] = fma(f[a][3 * k + 2], vJ[b][3 * k + 2], v);
        }
        __syncthreads();
        // node k's share goes to the owned entry of its block (node order)
        if (t < 252) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double mk = Mk[k][ab];
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) acc[s4] += rel[k] == jr0 + 7 * s4 ? mk : 0.0;
            }
        }
    }
    // E[(I, a), (J, b)] into the banded super-block storage (D: diagonal
    // super-blocks, B: couplings below the diagonal; entries above it are the
    // transposes written by the workgroups of the later blocks)
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
        const int a = ab / 6, b = ab % 6, jr = jr0 + 7 * s4;
        if (t >= 252 || jr >= 27) break;
        const int jb[3] = {ib[0] + jr % 3 - 1, ib[1] + (jr / 3) % 3 - 1, ib[2] + jr / 9 - 1};
        if (jb[0] < 0 || jb[0] >= p.nb[0] || jb[1] < 0 || jb[1] >= p.nb[1] || jb[2] < 0 || jb[2] >= p.nb[2]) continue;
        const int J = jb[0] + p.nb[0] * (jb[1] + p.nb[1] * jb[2]);
        double* at = coarse_slot(D, B, p.P, p.K, p.m, p.perm[6 * I + a], p.perm[6 * J + b]);
        if (at) *at = acc[s4];
    }
}

__global__ void k_init_coarse(int K, int P, const int32_t* iperm, double* D) {
    // identity on the padding unknowns (positions holding no coarse unknown)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = K * P;
    if (i >= n || iperm[i] >= 0) return;
    const int k = i / P, r = i % P;
    D[((int64_t)k * P + r) * P + r] = 1.0;
}

__global__ void k_extract_diag(int K, int P, const double* D, double* ed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * P) return;
    const int k = i / P, r = i % P;
    ed[i] = D[((int64_t)k * P + r) * P + r];
}

// ------------------------------------------------------------------ solve
// y[r][i] = c[r][i] + alpha * sum_j M[i][j] x[r][j] over j in [lo(i), hi(i)):
// one wavefront per row (coalesced row stream, x from cache), four rows per
// workgroup, batched over blockIdx.y.  tri = 1: M lower triangular
// (j <= i); tri = 2: upper (j >= i); tri = 0: the column window
// [c0, c1).  Entries outside the range are stored zeros and are not read.
// The copies at the ends of the coarse solve ride along: batch io.dual_k is
// also written to io.y2, and with io.mu the results (of batch io.mu_k, or of
// every batch) are also scattered to natural order.
struct GemvIO {
    const int32_t* iperm;  // ordered position -> natural coarse index (-1: padding)
    int ncoarse;
    double* y2;            // second output for batch dual_k (null: none)
    int dual_k;
    double* mu;            // scatter target [nrhs][ncoarse] (null: none)
    int mu_k;              // batch to scatter (-1: every batch)
    int qbase;             // position of row 0 of batch 0
    int qstride;           // positions from one batch to the next
    // batch 1's own column window [c0b, c1b) (if c1b > 0); with M2 (single
    // batch) a second product M2 x2 over that window added to the same rows
    int c0b, c1b;
    const void* M2;
    const double* x2;
};
// per-lane 16-byte loads of the streamed matrix: 2 FP64 or 4 FP32 elements
template <typename TM>
struct Lanes {
    static constexpr int N = 16 / sizeof(TM);
};
__device__ __forceinline__ void load_lane(const double* p, double v[2]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    v[0] = a.x;
    v[1] = a.y;
}
__device__ __forceinline__ void load_lane(const float* p, double v[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
}
// TM: element type of the streamed matrix (FP64, or the FP32 copies); x, c,
// y and the accumulation are FP64
template <typename TM>
__global__ __launch_bounds__(256) void k_gemv(int P, const TM* M, int64_t mstride, const double* x,
                                              int64_t xstride, const double* c, int64_t cstride, double alpha,
                                              double* y, int64_t ystride, int nrhs, int64_t vstride, int tri, int c0,
                                              int c1, GemvIO io) {
    constexpr int N = Lanes<TM>::N;
    const int kb = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= P) return;
    x += kb * xstride;
    double acc[4] = {0, 0, 0, 0};
    // acc += m[j0:j1] . xv[j0:j1] for every right-hand side
    auto window = [&](const TM* m, const double* xv, int j0, int j1) {
        // aligned groups of N (P, the block offsets and the vector strides are
        // multiples of 4); group members outside [j0, j1) count zero.  A chunk
        // is GU 16-byte loads per lane of the matrix (and the matching FP64
        // loads of the first right-hand side), all issued before the first is
        // used, so that a row window of up to 64 * N * GU = 1024 columns (every
        // chain step's window) costs one memory latency instead of one per
        // four loads.  The FP32 copies take half the matrix loads per chunk:
        // with eight, their widened values and the twice as many x loads held
        // 164 registers (three wavefronts per SIMD), and the copies streamed no
        // faster than FP64
        constexpr int GU = 1024 / (64 * N);
        for (int jj = (j0 & ~(N - 1)) + N * lane; jj < j1; jj += 64 * N * GU) {
            double mv[GU][N], xv0[GU][N];
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int j = jj + 64 * N * u;
                if (j < j1) {
                    load_lane(m + j, mv[u]);
#pragma unroll
                    for (int e = 0; e < N; e += 2) {
                        const double2 xx = *reinterpret_cast<const double2*>(xv + j + e);
                        xv0[u][e] = xx.x;
                        xv0[u][e + 1] = xx.y;
                    }
                }
#pragma unroll
                for (int e = 0; e < N; ++e)
                    if (j >= j1 || j + e < j0 || j + e >= j1) mv[u][e] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int j = jj + 64 * N * u;
                if (j < j1) {
#pragma unroll
                    for (int e = 0; e < N; ++e) acc[0] = fma(mv[u][e], xv0[u][e], acc[0]);
                }
            }
            for (int r = 1; r < nrhs; ++r) {
                const double* xr = xv + r * vstride;
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    const int j = jj + 64 * N * u;
                    if (j < j1) {
#pragma unroll
                        for (int e = 0; e < N; e += 2) {
                            const double2 xx = *reinterpret_cast<const double2*>(xr + j + e);
                            acc[r] = fma(mv[u][e], xx.x, acc[r]);
                            acc[r] = fma(mv[u][e + 1], xx.y, acc[r]);
                        }
                    }
                }
            }
        }
    };
    const bool own = kb == 1 && io.c1b > 0;
    const int j0 = tri == 2 ? row : (tri == 1 ? 0 : (own ? io.c0b : c0));
    const int j1 = tri == 1 ? row + 1 : (tri == 2 ? P : (own ? io.c1b : c1));
    window(M + kb * mstride + (int64_t)row * P, x, j0, j1);
    if (io.M2) window(static_cast<const TM*>(io.M2) + (int64_t)row * P, io.x2, io.c0b, io.c1b);
    for (int r = 0; r < nrhs; ++r) {
        double v = acc[r];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) {
            const int64_t o = r * vstride + row;
            const double out = (c ? c[kb * cstride + o] : 0.0) + alpha * v;
            y[kb * ystride + o] = out;
            if (io.y2 && kb == io.dual_k) io.y2[kb * ystride + o] = out;
            if (io.mu && (io.mu_k < 0 || kb == io.mu_k)) {
                const int nat = io.iperm[io.qbase + (int64_t)kb * io.qstride + row];
                if (nat >= 0) io.mu[(int64_t)r * io.ncoarse + nat] = out;
            }
        }
    }
}

__global__ void k_perm_in(int ncoarse, int npad, const int32_t* perm, const int32_t* iperm, int nrhs,
                          const double* G, double* gp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i < npad && iperm[i] < 0) gp[(int64_t)r * npad + i] = 0.0;  // padding position
    if (i >= ncoarse) return;
    gp[(int64_t)r * npad + perm[i]] = G[(int64_t)r * ncoarse + i];
}

__global__ void k_count(const int32_t* a, int n, int32_t* out) {
    __shared__ int sh[256];
    int s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += a[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int i = 0; i < 256; ++i) tot += sh[i];
        *out = tot;
    }
}

template <typename TM>
inline TM* blkptr(TM* base, int k, int P) { return base + (int64_t)k * P * P; }

}  // namespace

int coarse_alloc(Coarse& c, hipStream_t s) {
    const Blocks& b = c.blk;
    const int64_t PP = (int64_t)b.P * b.P;
    const int64_t npad = (int64_t)b.K * b.P;
    size_t bytes = PP * b.K * sizeof(double);
    double** arrs[] = {&c.D, &c.B, &c.Linv, &c.LinvT, &c.T, &c.U};
    for (double** a : arrs) {
        if (afd::dev_malloc((void**)a, bytes) != hipSuccess) {
            coarse_free(c);
            set_error("coarse: out of device memory");
            return AFD_E_OOM;
        }
    }
    AFD_HIP_TRY(afd::dev_malloc((void**)&c.Ediag, npad * sizeof(double)));
    AFD_HIP_TRY(afd::dev_malloc((void**)&c.work, PP * sizeof(double)));
    if (b.m >= 1 && b.K - 2 >= b.m) {  // the second chain of the factorisation (default priority)
        AFD_HIP_TRY(afd::dev_malloc((void**)&c.work2, PP * sizeof(double)));
        AFD_HIP_TRY(hipStreamCreateWithFlags(&c.s2, hipStreamNonBlocking));
        AFD_HIP_TRY(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
        AFD_HIP_TRY(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
    }
    AFD_HIP_TRY(afd::dev_malloc((void**)&c.dropped_dev, (npad + 1) * sizeof(int32_t)));
    AFD_HIP_TRY(afd::dev_malloc((void**)&c.gperm, 4 * npad * sizeof(double)));
    AFD_HIP_TRY(hipMemsetAsync(c.gperm, 0, 4 * npad * sizeof(double), s));  // padding positions stay zero
    AFD_HIP_TRY(afd::dev_malloc((void**)&c.xperm, 4 * npad * sizeof(double)));
    AFD_HIP_TRY(afd::dev_malloc((void**)&c.perm, b.ncoarse * sizeof(int32_t)));
    AFD_HIP_TRY(afd::dev_malloc((void**)&c.iperm, npad * sizeof(int32_t)));
    // ordering: axes of fewest blocks fastest (a banded matrix), then the
    // super-blocks in the two-ended order
    std::vector<int32_t> perm(b.ncoarse);
    const int a0 = b.perm[0], a1 = b.perm[1], a2 = b.perm[2];
    for (int bk = 0; bk < b.nb[2]; ++bk)
        for (int bj = 0; bj < b.nb[1]; ++bj)
            for (int bi = 0; bi < b.nb[0]; ++bi) {
                const int bb[3] = {bi, bj, bk};
                const int nat = bi + b.nb[0] * (bj + b.nb[1] * bk);
                const int ord = bb[a0] + b.nb[a0] * (bb[a1] + b.nb[a1] * bb[a2]);
                for (int m = 0; m < 6; ++m) perm[6 * nat + m] = twist_position(6 * ord + m, b.P, b.K, b.m);
            }
    AFD_HIP_TRY(hipMemcpyAsync(c.perm, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    c.iperm_host.assign(npad, -1);
    for (int i = 0; i < b.ncoarse; ++i) c.iperm_host[perm[i]] = i;
    AFD_HIP_TRY(hipMemcpyAsync(c.iperm, c.iperm_host.data(), npad * sizeof(int32_t), hipMemcpyHostToDevice, s));
    AFD_HIP_TRY(hipStreamSynchronize(s));
    return AFD_OK;
}

void coarse_free(Coarse& c) {
    double** arrs[] = {&c.D, &c.B, &c.Linv, &c.LinvT, &c.T, &c.U, &c.Ediag, &c.work, &c.work2, &c.gperm, &c.xperm};
    if (c.s2) (void)hipStreamDestroy(c.s2);
    if (c.ev_fork) (void)hipEventDestroy(c.ev_fork);
    if (c.ev_join) (void)hipEventDestroy(c.ev_join);
    c.s2 = nullptr;
    c.ev_fork = c.ev_join = nullptr;
    for (double** a : arrs)
        if (*a) {
            (void)afd::dev_free(*a);
            *a = nullptr;
        }
    float** arrs32[] = {&c.Linv32, &c.LinvT32, &c.T32, &c.U32};
    for (float** a : arrs32)
        if (*a) {
            (void)afd::dev_free(*a);
            *a = nullptr;
        }
    c.valid32 = false;
    if (c.dropped_dev) (void)afd::dev_free(c.dropped_dev);
    if (c.perm) (void)afd::dev_free(c.perm);
    if (c.iperm) (void)afd::dev_free(c.iperm);
    c.iperm = nullptr;
    c.dropped_dev = nullptr;
    c.perm = nullptr;
    c.valid = false;
}

int coarse_begin(Coarse& c, hipStream_t s) {
    const Blocks& b = c.blk;
    const int64_t PP = (int64_t)b.P * b.P;
    AFD_HIP_TRY(hipMemsetAsync(c.D, 0, PP * b.K * sizeof(double), s));
    AFD_HIP_TRY(hipMemsetAsync(c.B, 0, PP * b.K * sizeof(double), s));
    c.valid = false;
    c.valid32 = false;
    return AFD_OK;
}

__global__ void k_narrow(int64_t n, const double* a, float* b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

int coarse_make_f32(Coarse& c, hipStream_t s) {
    if (!c.valid) {
        set_error("coarse: FP32 copy requested before the factorisation");
        return AFD_E_INVALID_ARG;
    }
    if (c.valid32) return AFD_OK;
    const Blocks& b = c.blk;
    const int64_t n = (int64_t)b.P * b.P * b.K;
    float** dst[] = {&c.Linv32, &c.LinvT32, &c.T32, &c.U32};
    const double* src[] = {c.Linv, c.LinvT, c.T, c.U};
    for (int i = 0; i < 4; ++i) {
        if (!*dst[i] && afd::dev_malloc((void**)dst[i], n * sizeof(float)) != hipSuccess) {
            set_error("coarse: out of device memory for the FP32 copies");
            return AFD_E_OOM;
        }
        hipLaunchKernelGGL(k_narrow, dim3(2048), dim3(256), 0, s, n, src[i], *dst[i]);
    }
    AFD_HIP_TRY(hipGetLastError());
    c.valid32 = true;
    return AFD_OK;
}

int coarse_direct(Coarse& c, const Grid& g, const double* rho, const uint8_t* nmask, const double* ke576,
                  bool rigid, hipStream_t s) {
    const Blocks& b = c.blk;
    DirP p;
    p.n[0] = g.nx, p.n[1] = g.ny, p.n[2] = g.nz;
    for (int a = 0; a < 3; ++a) {
        p.b[a] = b.b[a];
        p.nb[a] = b.nb[a];
    }
    p.inv_scale = b.inv_scale;
    p.P = b.P;
    p.ncoarse = b.ncoarse;
    p.K = b.K;
    p.m = b.m;
    p.perm = c.perm;
    p.rho = rho;
    p.nm = nmask;
    p.ke = ke576;
    p.rigid = rigid ? 1 : 0;
    // largest element box over the blocks, per axis
    int64_t ebox = 1, nbox = 1;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        int mx = 0;
        for (int q = 0; q < b.nb[a]; ++q) {
            const int lo = q * b.b[a], hi = (q == b.nb[a] - 1) ? n[a] : lo + b.b[a] - 1;
            mx = std::max(mx, std::min(hi, n[a] - 1) - std::max(lo - 1, 0) + 1);
        }
        ebox *= mx;
        nbox *= mx + 1;
    }
    const int64_t lds = ebox * 8 + ((nbox + 7) / 8) * 8;
    if (lds <= 48 * 1024)
        hipLaunchKernelGGL(k_coarse_direct<true>, dim3(b.nblk), dim3(256), (size_t)lds, s, p, c.D, c.B);
    else
        hipLaunchKernelGGL(k_coarse_direct<false>, dim3(b.nblk), dim3(256), 0, s, p, c.D, c.B);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int coarse_scatter_probe(Coarse& c, const double* G, int color, int mode, hipStream_t s) {
    const Blocks& b = c.blk;
    ScatP p;
    for (int a = 0; a < 3; ++a) p.nb[a] = b.nb[a];
    p.P = b.P;
    p.ncoarse = b.ncoarse;
    p.K = b.K;
    p.m = b.m;
    p.perm = c.perm;
    hipLaunchKernelGGL(k_scatter_probe, dim3((b.ncoarse + 255) / 256), dim3(256), 0, s, p, G, color, mode, c.D, c.B);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int coarse_factor(Coarse& c, hipStream_t s) {
    const Blocks& b = c.blk;
    const int P = b.P, K = b.K;
    const int64_t PP = (int64_t)P * P;
    const int npad = K * P;
    hipLaunchKernelGGL(k_init_coarse, dim3((npad + 255) / 256), dim3(256), 0, s, K, P, c.iperm, c.D);
    hipLaunchKernelGGL(k_extract_diag, dim3((npad + 255) / 256), dim3(256), 0, s, K, P, c.D, c.Ediag);
    AFD_HIP_TRY(hipMemsetAsync(c.Linv, 0, PP * K * sizeof(double), s));
    AFD_HIP_TRY(hipMemsetAsync(c.T, 0, PP * K * sizeof(double), s));
    AFD_HIP_TRY(hipMemsetAsync(c.U, 0, PP * K * sizeof(double), s));
    // The coupling block B_k = E(k+1, k) is zero outside its first w rows and
    // last w columns (half bandwidth w <= P), and so is C_k = B_k Linv_k^T
    // (Linv_k lower triangular); the Schur update then touches only the
    // leading w x w corner of D_{k+1}, T_k = Linv_k C_{k-1} only its last w
    // columns and U_k = Linv_k^T C_k^T only its first w columns.
    //   In the two-ended order (twist_position) position m starts chain B and
    // has no predecessor; the middle (position K-1) is also coupled to chain
    // A's end (position m-1) by X = E(K-1, m-1), held in B[m-1], which is zero
    // outside its LAST w rows and last w columns: C_X = X Linv_{m-1}^T has the
    // same window, its Schur update touches the trailing w x w corner of the
    // middle block, T_X = Linv_{K-1} C_X (kept in T[m], free since position m
    // has no predecessor) its last w columns, and U_X = Linv_{m-1}^T C_X^T
    // (kept in U[m-1]) its last w columns.
    const int w = std::min(b.w, P), o = P - w;
    const int m = b.m;
    double* Cx = m >= 1 ? blkptr(c.B, m - 1, P) + (int64_t)o * P + o : nullptr;  // C_X[o:P, o:P]
    // one position: Schur update(s), Cholesky, inverse, chain matrices
    auto position = [&](int k, hipStream_t st, double* work) -> int {
        double* Dk = blkptr(c.D, k, P);
        double* Li = blkptr(c.Linv, k, P);
        const bool pred = k > 0 && k != m;        // coupled to position k - 1
        const bool mid_x = k == K - 1 && m >= 1;  // the middle, also coupled to position m - 1
        if (pred) {  // D_k[0:w, 0:w] -= C_{k-1} C_{k-1}^T  (C stored in B[k-1])
            const double* Ck = blkptr(c.B, k - 1, P) + o;
            AFD_TRY(gemm(w, w, w, -1.0, Ck, P, 0, Ck, P, 1, 1.0, Dk, P, st));
        }
        if (mid_x)  // D_k[o:P, o:P] -= C_X C_X^T
            AFD_TRY(gemm(w, w, w, -1.0, Cx, P, 0, Cx, P, 1, 1.0, Dk + (int64_t)o * P + o, P, st));
        // dense blocked Cholesky of D_k, tile inverses into Linv's diagonal tiles
        for (int j0 = 0; j0 < P; j0 += NB) {
            const int nb = std::min(NB, P - j0);
            hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(256), 0, st, Dk, Li, P, j0, nb, c.Ediag + (int64_t)k * P,
                               c.dropped_dev + (int64_t)k * P);
            const int rows = P - j0 - nb;
            if (rows > 0) {
                hipLaunchKernelGGL(k_panel, dim3((rows + 63) / 64), dim3(256), 0, st, Dk, Li, P, j0, nb);
                AFD_TRY(gemm(rows, rows, nb, -1.0, Dk + (int64_t)(j0 + nb) * P + j0, P, 0,
                             Dk + (int64_t)(j0 + nb) * P + j0, P, 1, 1.0, Dk + (int64_t)(j0 + nb) * P + j0 + nb, P,
                             st));
            }
        }
        AFD_HIP_TRY(hipGetLastError());
        // Linv by recursive doubling: the diagonal tiles hold the tile
        // inverses; at block size sz every pair of neighbouring blocks A =
        // [a, a + sz), C = [a + sz, a + 2 sz) (the last one possibly shorter)
        // gets its off-diagonal block of the inverse, -C^-1 (L_CA A^-1), so
        // the pairs become the inverted blocks of size 2 sz.  The pairs of a
        // level are independent: two batched products per level (plus two
        // for a short last pair) instead of a chain of tile rows
        for (int sz = NB; sz < P; sz *= 2) {
            const int full = P / (2 * sz);                      // pairs with C of full size
            const int64_t step = (int64_t)2 * sz * P + 2 * sz;  // from one pair's blocks to the next
            // T_p = L[a+sz : a+2sz, a : a+sz] A^-1 into work (sz x sz each)
            AFD_TRY(gemm_batched(full, sz, sz, sz, 1.0, Dk + (int64_t)sz * P, P, step, Li, P, step, 0.0, work, sz,
                                 (int64_t)sz * sz, st));
            // X_CA = -C^-1 T_p
            AFD_TRY(gemm_batched(full, sz, sz, sz, -1.0, Li + (int64_t)sz * P + sz, P, step, work, sz,
                                 (int64_t)sz * sz, 0.0, Li + (int64_t)sz * P, P, step, st));
            const int a = full * 2 * sz, sc = P - a - sz;  // a shorter last pair
            if (sc > 0) {
                double* Tl = work + (int64_t)full * sz * sz;
                AFD_TRY(gemm(sc, sz, sz, 1.0, Dk + (int64_t)(a + sz) * P + a, P, 0, Li + (int64_t)a * P + a, P, 0, 0.0,
                             Tl, sz, st));
                AFD_TRY(gemm(sc, sz, sc, -1.0, Li + (int64_t)(a + sz) * P + a + sz, P, 0, Tl, sz, 0, 0.0,
                             Li + (int64_t)(a + sz) * P + a, P, st));
            }
        }
        hipLaunchKernelGGL(k_zero_dropped, dim3((P + 255) / 256, P), dim3(256), 0, st, Li, P,
                           c.dropped_dev + (int64_t)k * P);
        hipLaunchKernelGGL(k_transpose, dim3((P + 31) / 32, (P + 31) / 32), dim3(32, 8), 0, st, P, Li,
                           blkptr(c.LinvT, k, P));
        if (pred) {  // T_k[:, o:P] = Linv_k[:, 0:w] C_{k-1}[0:w, o:P]
            AFD_TRY(gemm(P, w, w, 1.0, Li, P, 0, blkptr(c.B, k - 1, P) + o, P, 0, 0.0, blkptr(c.T, k, P) + o, P, st));
        }
        if (mid_x)  // T_X[:, o:P] = Linv_k[:, o:P] C_X[o:P, o:P], into T[m]
            AFD_TRY(gemm(P, w, w, 1.0, Li + o, P, 0, Cx, P, 0, 0.0, blkptr(c.T, m, P) + o, P, st));
        if (k == m - 1) {
            // C_X = X[o:P, o:P] Linv_k[o:P, o:P]^T (in work, then back into B[m-1]);
            // U_X[:, o:P] = Linv_k[o:P, :]^T C_X^T, into U[m-1]
            AFD_TRY(gemm(w, w, w, 1.0, Cx, P, 0, Li + (int64_t)o * P + o, P, 1, 0.0, work, P, st));
            AFD_HIP_TRY(hipMemcpy2DAsync(Cx, P * sizeof(double), work, P * sizeof(double), w * sizeof(double), w,
                                         hipMemcpyDeviceToDevice, st));
            AFD_TRY(gemm(P, w, w, 1.0, Li + (int64_t)o * P, P, 1, Cx, P, 1, 0.0, blkptr(c.U, k, P) + o, P, st));
        } else if (k < K - 1) {
            // C_k[0:w, o:P] = B_k[0:w, o:P] Linv_k[o:P, o:P]^T (in work, then back into B[k])
            double* Bk = blkptr(c.B, k, P);
            AFD_TRY(gemm(w, w, w, 1.0, Bk + o, P, 0, Li + (int64_t)o * P + o, P, 1, 0.0, work, P, st));
            AFD_HIP_TRY(hipMemcpy2DAsync(Bk + o, P * sizeof(double), work, P * sizeof(double), w * sizeof(double), w,
                                         hipMemcpyDeviceToDevice, st));
            // U_k[:, 0:w] = Linv_k[o:P, :]^T C_k[0:w, o:P]^T
            AFD_TRY(gemm(P, w, w, 1.0, Li + (int64_t)o * P, P, 1, Bk + o, P, 1, 0.0, blkptr(c.U, k, P), P, st));
        }
        return AFD_OK;
    };
    // chains A (positions 0..m-1) and B (m..K-2) are independent until the
    // middle: B runs on a second stream (its own work buffer) beside A
    const bool two = m >= 1 && K - 2 >= m && c.s2 && c.work2;
    if (two) {
        AFD_HIP_TRY(hipEventRecord(c.ev_fork, s));
        AFD_HIP_TRY(hipStreamWaitEvent(c.s2, c.ev_fork, 0));
        for (int q = 0; q < std::max(m, K - 1 - m); ++q) {  // enqueued alternately, so both start at once
            if (q < m) AFD_TRY(position(q, s, c.work));
            if (m + q <= K - 2) AFD_TRY(position(m + q, c.s2, c.work2));
        }
        AFD_HIP_TRY(hipEventRecord(c.ev_join, c.s2));
        AFD_HIP_TRY(hipStreamWaitEvent(s, c.ev_join, 0));
    } else {
        for (int k = 0; k < K - 1; ++k) AFD_TRY(position(k, s, c.work));
    }
    AFD_TRY(position(K - 1, s, c.work));
    hipLaunchKernelGGL(k_count, dim3(1), dim3(256), 0, s, c.dropped_dev, npad, c.dropped_dev + npad);
    AFD_HIP_TRY(hipGetLastError());
    int32_t nd = 0;
    AFD_HIP_TRY(hipMemcpyAsync(&nd, c.dropped_dev + npad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    AFD_HIP_TRY(hipStreamSynchronize(s));
    c.dropped = nd;
    c.valid = true;
    c.valid32 = false;
    if (nd >= b.ncoarse) {
        set_error("coarse: every pivot dropped");
        return AFD_E_COARSE_SINGULAR;
    }
    return AFD_OK;
}

template <typename TM>
int coarse_solve_t(Coarse& c, int nrhs, const double* G, double* MU, hipStream_t s, const TM* Linv, const TM* LinvT,
                   const TM* T, const TM* U, bool g_in_perm) {
    const Blocks& b = c.blk;
    const int P = b.P, K = b.K;
    const int64_t PP = (int64_t)P * P;
    const int npad = K * P;
    // coupling blocks E(k, k-1) are zero outside their last w columns, E(k, k+1)
    // outside their first w columns (half bandwidth w <= P), so the chain
    // products only stream that window.  Two-ended order (twist_position):
    // chains A (positions 0..m-1) and B (m..K-2) run side by side, one launch
    // per pair of steps, and meet the middle (K-1), which also couples to
    // position m-1 through T_X (in T[m]) and U_X (in U[m-1]), last-w windows;
    // the middle's two products share one launch each way.
    const int w = std::min(b.w, P), o = P - w;
    const int m = b.m;
    const int la = std::max(m - 1, 0), lb = std::max(K - 2 - m, 0);  // chain steps of A and B
    const unsigned rb = (unsigned)((P + 3) / 4);
    GemvIO none{c.iperm, b.ncoarse, nullptr, -1, nullptr, -1, 0, P};
    // one launch of chain steps: positions pa (if >= 0) and pb (if >= 0), each
    // v[pos] -= M[pos] v[pos + from] over the window [c0, c1), in place
    auto chain = [&](const TM* M, double* v, int pa, int pb, int from, int c0, int c1, GemvIO io) {
        const int p0 = pa >= 0 ? pa : pb;
        const int nb = (pa >= 0 && pb >= 0) ? 2 : 1;
        const int64_t d = nb == 2 ? (int64_t)(pb - pa) : 0;
        io.qbase = p0 * P;
        io.qstride = (int)(d * P);
        hipLaunchKernelGGL(k_gemv<TM>, dim3(rb, nb), dim3(256), 0, s, P, M + (int64_t)p0 * PP, d * PP,
                           v + (int64_t)(p0 + from) * P, d * P, v + (int64_t)p0 * P, d * P, -1.0, v + (int64_t)p0 * P,
                           d * P, nrhs, (int64_t)npad, 0, c0, c1, io);
    };

    // x_k = Linv_k g_k, all positions (g in the banded ordering; padding
    // positions of gperm are zero: set at allocation and by k_perm_in, and the
    // solve leaves them zero since padding rows of the factor are identity)
    if (!g_in_perm)
        hipLaunchKernelGGL(k_perm_in, dim3((npad + 255) / 256, nrhs), dim3(256), 0, s, b.ncoarse, npad, c.perm,
                           c.iperm, nrhs, G, c.gperm);
    hipLaunchKernelGGL(k_gemv<TM>, dim3(rb, K), dim3(256), 0, s, P, Linv, PP, c.gperm, (int64_t)P,
                       (const double*)nullptr, (int64_t)0, 1.0, c.xperm, (int64_t)P, nrhs, (int64_t)npad, 1, 0, P,
                       none);
    // x_k -= T_k x_{k-1} along both chains, then the middle
    for (int q = 1; q <= std::max(la, lb); ++q)
        chain(T, c.xperm, q <= la ? q : -1, q <= lb ? m + q : -1, -1, o, P, none);
    if (K >= 2) {  // the middle: x_{K-1} -= T_{K-1} x_{K-2} + T_X x_{m-1}, one launch
        GemvIO mid = none;
        if (m >= 1) {
            mid.M2 = blkptr(T, m, P);
            mid.x2 = c.xperm + (int64_t)(m - 1) * P;
            mid.c0b = o, mid.c1b = P;
        }
        chain(T, c.xperm, -1, K - 1, -1, o, P, mid);
    }
    // mu_k = Linv_k^T x_k, all positions; mu_{K-1} is final (scattered)
    GemvIO last = none;
    last.mu = MU;
    last.mu_k = K - 1;
    hipLaunchKernelGGL(k_gemv<TM>, dim3(rb, K), dim3(256), 0, s, P, LinvT, PP, c.xperm, (int64_t)P,
                       (const double*)nullptr, (int64_t)0, 1.0, c.gperm, (int64_t)P, nrhs, (int64_t)npad, 2, 0, P,
                       last);
    // mu_k -= U_k mu_{k+1} away from the middle, scattered to natural order as produced
    GemvIO sc = none;
    sc.mu = MU;
    if (K >= 2) {  // from the middle: mu_{K-2} -= U_{K-2} mu_{K-1} and mu_{m-1} -= U_X mu_{K-1}, one launch
        const int nb = m >= 1 ? 2 : 1;
        const int64_t d = m >= 1 ? (int64_t)(m - 1) - (K - 2) : 0;  // position step to the second output
        GemvIO hd = sc;
        hd.qbase = (K - 2) * P;
        hd.qstride = (int)(d * P);
        hd.c0b = o, hd.c1b = P;  // U_X's window
        hipLaunchKernelGGL(k_gemv<TM>, dim3(rb, nb), dim3(256), 0, s, P, blkptr(U, K - 2, P), d * PP,
                           c.gperm + (int64_t)(K - 1) * P, (int64_t)0, c.gperm + (int64_t)(K - 2) * P, d * P, -1.0,
                           c.gperm + (int64_t)(K - 2) * P, d * P, nrhs, (int64_t)npad, 0, 0, w, hd);
    }
    for (int q = 1; q <= std::max(la, lb); ++q)
        chain(U, c.gperm, q <= la ? m - 1 - q : -1, q <= lb ? K - 2 - q : -1, 1, 0, w, sc);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int coarse_solve(Coarse& c, int nrhs, const double* G, double* MU, hipStream_t s, bool f32, bool g_in_perm) {
    if (f32) {
        if (!c.valid32) {
            set_error("coarse: FP32 solve without the FP32 copies");
            return AFD_E_INVALID_ARG;
        }
        return coarse_solve_t<float>(c, nrhs, G, MU, s, c.Linv32, c.LinvT32, c.T32, c.U32, g_in_perm);
    }
    return coarse_solve_t<double>(c, nrhs, G, MU, s, c.Linv, c.LinvT, c.T, c.U, g_in_perm);
}

int coarse_to_dense_host(Coarse& c, double* E, hipStream_t s) {
    const Blocks& b = c.blk;
    const int P = b.P, K = b.K, n = b.ncoarse;
    const int64_t PP = (int64_t)P * P;
    std::vector<double> D(PP * K), B(PP * K);
    std::vector<int32_t> perm(n);
    AFD_HIP_TRY(hipMemcpyAsync(D.data(), c.D, PP * K * sizeof(double), hipMemcpyDeviceToHost, s));
    AFD_HIP_TRY(hipMemcpyAsync(B.data(), c.B, PP * K * sizeof(double), hipMemcpyDeviceToHost, s));
    AFD_HIP_TRY(hipMemcpyAsync(perm.data(), c.perm, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    AFD_HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int pi = perm[i], pj = perm[j];
            const double* at = coarse_slot(D.data(), B.data(), P, K, b.m, pi, pj);
            if (!at) at = coarse_slot(D.data(), B.data(), P, K, b.m, pj, pi);  // kept as the transpose
            E[(int64_t)i * n + j] = at ? *at : 0.0;
        }
    return AFD_OK;
}

}  // namespace afd
