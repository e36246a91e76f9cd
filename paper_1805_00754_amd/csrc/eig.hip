// Leading eigenvectors of a symmetric positive semi-definite c x c Gram matrix,
// one work-group per matrix, entirely in LDS (c <= 128 in FP64: 129 KiB).
//
// This is the first stage of every rank-k SVD the method takes (the block
// SVD of the storage phase and the SVD of a query's stacked matrix):
//   1. G  <- sum of the problem's Gram terms (fixed order): partial Grams of
//            a block's row chunks, or, for a query, the Gram-tree nodes that
//            cover its whole blocks plus the Grams of its Partial-SVD rows;
//   2. L  <- Cholesky factor of G + s I, s = 4 (c+1) eps tr(G).  The shift
//            keeps the factorisation alive on rank-deficient input and does
//            not move the eigenvectors of G;
//   3. one-sided Jacobi on the columns of L (parallel round-robin ordering,
//      TPP lanes per column pair, column slices held in registers).  When the
//      columns are orthogonal, L J = Q Sigma with Q the eigenvectors of
//      L L^T = G + s I, so no rotation is accumulated;
//   4. V_k <- the kk columns of largest norm, normalised (ties by index).
// The eigenvalues found here are discarded: the second stage recomputes the
// singular values from the data with relative accuracy (finalize kernel).
#include "zs_internal.h"

namespace zs {
namespace {

__device__ __forceinline__ void rr_pair(int step, int pi, int N, int &p, int &q)
{
    // Circle method: index 0 is fixed, indices 1..N-1 rotate by one per step.
    const int m = N - 1;
    if (pi == 0) {
        p = 0;
        q = 1 + (step % m);
    } else {
        p = 1 + ((pi + step) % m);
        q = 1 + ((m - pi + step) % m);
    }
}

template <int NMAX>
__global__ __launch_bounds__(kThreads) void eig_kernel(int c, int k, const Prob *__restrict__ probs,
                                                       const double *const *__restrict__ gsrc,
                                                       const double *const *__restrict__ msrc,
                                                       double *__restrict__ Vk,
                                                       int *__restrict__ conv_flag)
{
    constexpr int LDX = NMAX + 1;
    constexpr int NP = NMAX / 2;
    constexpr int TPP0 = kThreads / NP;
    constexpr int TPP = TPP0 < NMAX / 2 ? TPP0 : NMAX / 2;
    constexpr int ELEMS = (NMAX + TPP - 1) / TPP;
    constexpr int MR = 8;              // rows of a k x c block staged at a time
    extern __shared__ __align__(16) double smem[];
    double *X = smem;                  // column-major, column j at X + j * LDX
    double *nu = X + NMAX * LDX;       // column norms
    double *Rs = nu + NMAX;            // MR x c staging of row blocks
    __shared__ int rot_count;
    __shared__ double sh_shift, sh_tr;

    const Prob P = probs[blockIdx.x];
    const int tid = threadIdx.x;

    // 1. G = sum of the problem's c x c Gram terms (fixed order) plus the
    //    Grams R^T R of its k x c row blocks.  Symmetric: column-major == row-major.
    for (int e = tid; e < c * c; e += kThreads) {
        const int i = e / c, j = e % c;
        double s = 0.0;
        for (int g = 0; g < P.ng; ++g) s += gsrc[P.g0 + g][e];
        X[j * LDX + i] = s;
    }
    for (int m = 0; m < P.nm; ++m) {
        const double *R = msrc[P.m0 + m];
        for (int r0 = 0; r0 < k; r0 += MR) {
            const int nr = min(MR, k - r0);
            __syncthreads();
            for (int e = tid; e < nr * c; e += kThreads) Rs[e] = R[(int64_t)r0 * c + e];
            __syncthreads();
            for (int e = tid; e < c * c; e += kThreads) {
                const int i = e / c, j = e % c;
                double s = X[j * LDX + i];
                for (int r = 0; r < nr; ++r) s = fma(Rs[r * c + i], Rs[r * c + j], s);
                X[j * LDX + i] = s;
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0;
        for (int i = 0; i < c; ++i) tr += X[i * LDX + i];
        double s = 4.0 * (c + 1) * __DBL_EPSILON__ * tr;
        if (!(s > 0.0)) s = 1.0;               // zero (or invalid) matrix
        sh_shift = s;
        sh_tr = tr > 0.0 ? tr : 0.0;
    }
    __syncthreads();
    const double shift = sh_shift;
    for (int i = tid; i < c; i += kThreads) X[i * LDX + i] += shift;
    __syncthreads();

    // 2. Cholesky G + s I = L L^T, in place, lower triangle, column-major.
    for (int j = 0; j < c; ++j) {
        if (tid == 0) {
            double d = X[j * LDX + j];
            if (!(d > 0.5 * shift)) d = shift;   // clamp: rounding pushed the pivot down
            X[j * LDX + j] = sqrt(d);
        }
        __syncthreads();
        const double ljj = X[j * LDX + j];
        for (int i = j + 1 + tid; i < c; i += kThreads) X[j * LDX + i] /= ljj;
        __syncthreads();
        const int n2 = c - j - 1;
        for (int e = tid; e < n2 * n2; e += kThreads) {
            const int jj = j + 1 + e / n2, i = j + 1 + e % n2;
            if (i >= jj) X[jj * LDX + i] -= X[j * LDX + i] * X[j * LDX + jj];
        }
        __syncthreads();
    }
    for (int e = tid; e < c * c; e += kThreads) {
        const int j = e / c, i = e % c;
        if (i < j) X[j * LDX + i] = 0.0;
    }
    __syncthreads();

    // 3. One-sided Jacobi on the columns of L.
    const double tol = (double)c * __DBL_EPSILON__;
    const double fro2 = sh_tr + c * shift;     // ||L||_F^2 = tr(L L^T) = tr(G + s I)
    const double floor2 = ((double)c * __DBL_EPSILON__) * ((double)c * __DBL_EPSILON__) * fro2;
    const int N = (c + 1) & ~1;
    const int pi = tid / TPP, lane = tid % TPP;
    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        if (tid == 0) rot_count = 0;
        __syncthreads();
        for (int step = 0; step < N - 1; ++step) {
            if (pi < N / 2) {
                int p, q;
                rr_pair(step, pi, N, p, q);
                const bool act = (p < c) && (q < c);
                double xp[ELEMS], xq[ELEMS];
                double a = 0.0, b2 = 0.0, g = 0.0;
#pragma unroll
                for (int e = 0; e < ELEMS; ++e) {
                    const int row = lane + e * TPP;
                    const bool in = act && row < c;
                    xp[e] = in ? X[p * LDX + row] : 0.0;
                    xq[e] = in ? X[q * LDX + row] : 0.0;
                    a = fma(xp[e], xp[e], a);
                    b2 = fma(xq[e], xq[e], b2);
                    g = fma(xp[e], xq[e], g);
                }
#pragma unroll
                for (int off = TPP / 2; off >= 1; off >>= 1) {
                    a += __shfl_xor(a, off, 64);
                    b2 += __shfl_xor(b2, off, 64);
                    g += __shfl_xor(g, off, 64);
                }
                const bool rot = act && a > floor2 && b2 > floor2 &&
                                 fabs(g) > tol * sqrt(a) * sqrt(b2);
                if (rot) {
                    const double zeta = (b2 - a) / (2.0 * g);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + t * t);
                    const double sn = cs * t;
#pragma unroll
                    for (int e = 0; e < ELEMS; ++e) {
                        const int row = lane + e * TPP;
                        if (row < c) {
                            X[p * LDX + row] = cs * xp[e] - sn * xq[e];
                            X[q * LDX + row] = sn * xp[e] + cs * xq[e];
                        }
                    }
                    if (lane == 0) atomicAdd(&rot_count, 1);
                }
            }
            __syncthreads();
        }
        const int rc = rot_count;
        __syncthreads();
        if (rc == 0) break;
    }
    if (sweep == kMaxSweeps && tid == 0) atomicOr(conv_flag, 1);

    // 4. Normalised columns of largest norm.
    for (int j = tid; j < c; j += kThreads) {
        double s = 0.0;
        for (int i = 0; i < c; ++i) s = fma(X[j * LDX + i], X[j * LDX + i], s);
        nu[j] = sqrt(s);
    }
    __syncthreads();
    const int kk = P.kk;
    double *out = Vk + (int64_t)blockIdx.x * c * kMaxK;
    for (int j = tid; j < c; j += kThreads) {
        const double nj = nu[j];
        int pos = 0;
        for (int i = 0; i < c; ++i) {
            const double ni = nu[i];
            pos += (ni > nj) || (ni == nj && i < j);
        }
        if (pos < kk) {
            const double inv = nj > 0.0 ? 1.0 / nj : 0.0;
            for (int row = 0; row < c; ++row) out[row * kk + pos] = X[j * LDX + row] * inv;
        }
    }
}

template <int NMAX>
hipError_t run_eig(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                   const double *const *msrc, double *Vk, int *conv_flag, hipStream_t stream)
{
    const size_t lds = (size_t)(NMAX * (NMAX + 1) + NMAX + 8 * NMAX) * sizeof(double);
    static size_t cur = 0;
    hipError_t e = ensure_lds((const void *)eig_kernel<NMAX>, lds, cur);
    if (e != hipSuccess) return e;
    eig_kernel<NMAX><<<nprob, kThreads, lds, stream>>>(c, k, probs, gsrc, msrc, Vk, conv_flag);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eig(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                      const double *const *msrc, double *Vk, int *conv_flag, hipStream_t stream)
{
    if (nprob <= 0) return hipSuccess;
    if (c > kMaxC) return hipErrorInvalidValue;
    timing_begin("eig", stream);
    hipError_t e;
    if (c <= 16) e = run_eig<16>(c, k, probs, nprob, gsrc, msrc, Vk, conv_flag, stream);
    else if (c <= 32) e = run_eig<32>(c, k, probs, nprob, gsrc, msrc, Vk, conv_flag, stream);
    else if (c <= 64) e = run_eig<64>(c, k, probs, nprob, gsrc, msrc, Vk, conv_flag, stream);
    else e = run_eig<128>(c, k, probs, nprob, gsrc, msrc, Vk, conv_flag, stream);
    timing_end("eig", stream);
    return e;
}

}  // namespace zs
