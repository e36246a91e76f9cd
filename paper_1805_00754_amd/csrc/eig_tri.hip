// Leading eigenvectors of a symmetric positive semi-definite c x c Gram matrix
// by tridiagonalisation, one work-group per matrix, in LDS (c <= 128).
//
// First stage of every rank-k SVD of the method (the block SVDs of the
// storage phase and the SVD of each query's stacked matrix).  Only the span of
// the kk leading eigenvectors is used: the Rayleigh-Ritz stage that follows
// recomputes the singular values from the data with relative accuracy.
//
//   1. G <- the problem's Gram terms (fixed order), as in the Jacobi variant.
//   2. Householder tridiagonalisation Q^T G Q = T (Golub & Van Loan 8.3.1),
//      each reflector vector packed into matrix rows the reduction is done with.
//   3. The kk largest eigenvalues of T by multisection on Sturm counts
//      (groups of up to 64 threads per eigenvalue).
//   4. Eigenvectors of T by inverse iteration (tridiagonal LU with partial
//      pivoting, two solves, one thread per cluster of eigenvalues closer
//      than 1e-9 ||T||, Gram-Schmidt inside a cluster: the approach of
//      LAPACK's stein).
//   5. Back-transformation x = Q z, then two passes of classical Gram-Schmidt
//      over the kk vectors (a vector that collapses is replaced by the next
//      unit vector, which can only happen inside a degenerate eigenspace).
// The total work is O(c^3) with a small constant, against O(50 c^3) for
// one-sided Jacobi.
#include "zs_internal.h"

namespace zs {
namespace {

constexpr int NTH = 1024;                 // threads of the eigen-solver work-group
constexpr int kWaves = NTH / 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic start vector in (-1, 1) for inverse iteration.
__device__ __forceinline__ double start_value(int i, int g, int attempt)
{
    uint32_t x = (uint32_t)i * 2654435761u ^ (uint32_t)(g + 1 + 97 * attempt) * 2246822519u;
    x ^= x >> 15;
    x *= 2246822519u;
    x ^= x >> 13;
    x *= 3266489917u;
    x ^= x >> 16;
    return (double)(x & 0xFFFFFF) / 8388608.0 - 1.0;
}

// LDS layout of the solver (doubles): d, e, e2, tau (NMAX each), lam (kMaxK),
// then one region of REGION doubles.  The region holds the matrix during the
// tridiagonal reduction; the reduction packs each Householder vector into rows
// it no longer needs, so that afterwards the region holds, in order: the
// packed vectors, the eigenvector block Z (c x kk) and the inverse-iteration
// arrays.  All data stays in LDS between phases; global memory is written once.
template <int NMAX>
struct TriLayout {
    static constexpr int LDA = NMAX + 1;
    static constexpr int AREA = NMAX * LDA;
    static constexpr int HPMAX = (NMAX - 1) * NMAX / 2;             // packed vectors
    static constexpr int KZ = NMAX < kMaxK ? NMAX : kMaxK;           // largest kk
    static constexpr int NEED = HPMAX + NMAX * KZ + 4 * NMAX * 4;     // >= 4 solver threads
    static constexpr int R0 = AREA + 1536;
    static constexpr int REGION = R0 > NEED ? R0 : NEED;
    static constexpr size_t bytes() { return (size_t)(4 * NMAX + kMaxK + REGION) * sizeof(double); }
};

template <int NMAX>
__global__ __launch_bounds__(NTH) void eig_tri_kernel(int c, int k, const Prob *__restrict__ probs,
                                                      const double *const *__restrict__ gsrc,
                                                      const double *const *__restrict__ msrc,
                                                      double *__restrict__ Vk)
{
    using L = TriLayout<NMAX>;
    constexpr int LDA = L::LDA;
    constexpr int MR = 8;
    extern __shared__ __align__(16) double smem[];
    double *d = smem;
    double *e = d + NMAX;
    double *e2 = e + NMAX;
    double *tau = e2 + NMAX;
    double *lam = tau + NMAX;                      // kMaxK
    double *A = lam + kMaxK;                       // region: matrix, row-major A[i * LDA + j]
    double *scr = A + L::AREA;                     // tail of the region (phases 1-3)
    __shared__ double sh_a, sh_b, sh_tnorm, sh_pivmin;
    __shared__ double glo[kMaxK], ghi[kMaxK];
    __shared__ int cl_start[kMaxK + 1];
    __shared__ int sh_ncl, sh_done;

    const Prob P = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int kk = P.kk;
    double *out = Vk + (int64_t)blockIdx.x * c * kMaxK;   // c x kk, row-major
    // packed Householder vector j starts at hoff(j); its entry 0 is 1
    auto hoff = [c](int j) { return j * (c - 1) - j * (j - 1) / 2; };

    // ---- 1. G ------------------------------------------------------------------
    for (int q = tid; q < c * c; q += NTH) {
        double s = 0.0;
        for (int g = 0; g < P.ng; ++g) s += gsrc[P.g0 + g][q];
        A[(q / c) * LDA + q % c] = s;
    }
    for (int m = 0; m < P.nm; ++m) {
        const double *R = msrc[P.m0 + m];
        double *Rs = scr;                          // MR x c
        for (int r0 = 0; r0 < k; r0 += MR) {
            const int nr = min(MR, k - r0);
            __syncthreads();
            for (int q = tid; q < nr * c; q += NTH) Rs[q] = R[(int64_t)r0 * c + q];
            __syncthreads();
            for (int q = tid; q < c * c; q += NTH) {
                const int i = q / c, j = q % c;
                double s2 = A[i * LDA + j];
                for (int r = 0; r < nr; ++r) s2 = fma(Rs[r * c + i], Rs[r * c + j], s2);
                A[i * LDA + j] = s2;
            }
        }
    }
    __syncthreads();

    // ---- 2. tridiagonalisation (three barriers per reflector) -----------------------
    double *vsh = scr;
    double *psh = scr + NMAX;
    for (int j = 0; j + 2 < c; ++j) {
        const int n1 = c - j - 1;
        // Householder vector of A[j+1:, j]; every wave computes the scalars itself.
        double s = 0.0;
        for (int i = j + 2 + lane; i < c; i += 64) s = fma(A[i * LDA + j], A[i * LDA + j], s);
        s = wave_sum(s);
        const double alpha = A[(j + 1) * LDA + j];
        double t = 0.0, beta = alpha, scal = 0.0;
        if (s > 0.0) {
            const double mu = sqrt(alpha * alpha + s);
            beta = alpha <= 0.0 ? mu : -mu;
            t = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        if (tid == 0) {
            tau[j] = t;
            e[j] = beta;
            d[j] = A[j * LDA + j];
        }
        for (int i = tid; i < n1; i += NTH) vsh[i] = (i == 0) ? 1.0 : A[(j + 1 + i) * LDA + j] * scal;
        __syncthreads();
        // Pack v_j into rows <= j, which are no longer read (row j's diagonal was
        // taken above); the packed range ends before row j+1.
        for (int i = tid; i < n1; i += NTH) A[hoff(j) + i] = vsh[i];
        if (t == 0.0) {                            // uniform: nothing to annihilate
            __syncthreads();
            continue;
        }
        // p = t * A22 v: eight threads per row (all rows in one pass)
        {
            const int row = tid / 8, sub = tid % 8;
            double s0 = 0.0, s1 = 0.0;
            if (row < n1) {
                const double *ar = A + (j + 1 + row) * LDA + j + 1;
                int col = sub;
                for (; col + 8 < n1; col += 16) {
                    s0 = fma(ar[col], vsh[col], s0);
                    s1 = fma(ar[col + 8], vsh[col + 8], s1);
                }
                if (col < n1) s0 = fma(ar[col], vsh[col], s0);
            }
            double sum = s0 + s1;
            sum += __shfl_xor(sum, 4, 64);
            sum += __shfl_xor(sum, 2, 64);
            sum += __shfl_xor(sum, 1, 64);
            if (sub == 0 && row < n1) psh[row] = t * sum;
        }
        __syncthreads();
        // K = t/2 p.v, computed by every wave; A22 -= v w^T + w v^T with w = p - K v.
        // Thread (tr, ts) of a 32 x 32 grid keeps the v, w entries of its columns.
        double sk = 0.0;
        for (int i = lane; i < n1; i += 64) sk = fma(psh[i], vsh[i], sk);
        const double K = 0.5 * t * wave_sum(sk);
        const int tr = tid / 32, ts = tid % 32;
        double vc[4], wc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s2 = ts + 32 * u;
            vc[u] = s2 < n1 ? vsh[s2] : 0.0;
            wc[u] = s2 < n1 ? psh[s2] - K * vc[u] : 0.0;
        }
        for (int r = tr; r < n1; r += 32) {
            const double vr = vsh[r], wr = psh[r] - K * vr;
            double *ar = A + (j + 1 + r) * LDA + j + 1;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int s2 = ts + 32 * u;
                if (s2 < n1) ar[s2] -= vr * wc[u] + wr * vc[u];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (c >= 2) {
            d[c - 2] = A[(c - 2) * LDA + c - 2];
            e[c - 2] = A[(c - 1) * LDA + c - 2];
        }
        d[c - 1] = A[(c - 1) * LDA + c - 1];
        double gl = d[0], gu = d[0], emax2 = 0.0;
        for (int i = 0; i < c; ++i) {
            const double ei = i + 1 < c ? fabs(e[i]) : 0.0;
            const double em = i > 0 ? fabs(e[i - 1]) : 0.0;
            gl = fmin(gl, d[i] - ei - em);
            gu = fmax(gu, d[i] + ei + em);
            if (i + 1 < c) emax2 = fmax(emax2, e[i] * e[i]);
        }
        const double tn = fmax(fabs(gl), fabs(gu));
        const double pivmin = __DBL_MIN__ * fmax(1.0, emax2);
        sh_tnorm = tn;
        sh_pivmin = pivmin;
        sh_a = gl - 2.1 * tn * __DBL_EPSILON__ * c - 4.2 * pivmin;
        sh_b = gu + 2.1 * tn * __DBL_EPSILON__ * c + 4.2 * pivmin;
    }
    __syncthreads();                               // e[c - 2] was written by thread 0
    for (int i = tid; i + 1 < c; i += NTH) e2[i] = e[i] * e[i];
    __syncthreads();
    const double tnorm = sh_tnorm, pivmin = sh_pivmin;

    if (tnorm == 0.0) {                   // zero matrix: any orthonormal basis
        for (int q = tid; q < c * kk; q += NTH) out[q] = (q / kk == q % kk) ? 1.0 : 0.0;
        return;
    }

    // ---- 3. the kk largest eigenvalues: multisection on Sturm counts ---------------
    {
        const int G = min(NTH / kk, 64);
        const int grp = tid / G, mem = tid % G;
        const int m = c - 1 - grp;                 // ascending index of the wanted eigenvalue
        double *xs = scr;                          // G * kk <= NTH
        int *cs = reinterpret_cast<int *>(scr + NTH);
        if (tid < kk) {
            glo[tid] = sh_a;
            ghi[tid] = sh_b;
        }
        const double atol = 4.0 * __DBL_EPSILON__ * tnorm + 2.0 * pivmin;
        for (int it = 0; it < 80; ++it) {
            if (tid == 0) sh_done = 1;
            __syncthreads();
            if (grp < kk) {
                const double lo = glo[grp], hi = ghi[grp];
                const double x = lo + (hi - lo) * (double)(mem + 1) / (double)(G + 1);
                double q = d[0] - x;
                if (fabs(q) < pivmin) q = -pivmin;
                int cnt = q < 0.0;
                for (int i = 1; i < c; ++i) {
                    q = d[i] - x - e2[i - 1] / q;
                    if (fabs(q) < pivmin) q = -pivmin;
                    cnt += q < 0.0;
                }
                xs[tid] = x;
                cs[tid] = cnt;
            }
            __syncthreads();
            if (grp < kk && mem == 0) {
                double lo = glo[grp], hi = ghi[grp];
                for (int u = 0; u < G; ++u) {
                    if (cs[grp * G + u] <= m) {
                        lo = xs[grp * G + u];
                    } else {
                        hi = xs[grp * G + u];
                        break;
                    }
                }
                glo[grp] = lo;
                ghi[grp] = hi;
                if (hi - lo > atol) sh_done = 0;
            }
            __syncthreads();
            const int done = sh_done;
            __syncthreads();
            if (done) break;
        }
        if (tid < kk) lam[tid] = 0.5 * (glo[tid] + ghi[tid]);
    }
    __syncthreads();
    // clusters of consecutive eigenvalues closer than 1e-9 ||T||
    if (tid == 0) {
        int n = 0;
        cl_start[n++] = 0;
        for (int g = 1; g < kk; ++g)
            if (lam[g - 1] - lam[g] > 1e-9 * tnorm) cl_start[n++] = g;
        cl_start[n] = kk;
        sh_ncl = n;
    }
    __syncthreads();

    // ---- 4. inverse iteration: one thread per cluster, members in order ----------
    //      Z (c x kk) follows the packed vectors; each solver thread keeps four
    //      length-c arrays after Z, interleaved by thread (element i at i * NT + t).
    const int hp = c >= 3 ? hoff(c - 2) : 0;        // packed length
    double *Z = A + hp;
    {
        double *lu = Z + c * kk;
        const int NT = min((int)((A + L::REGION - lu) / (4 * c)), NTH);
        const int ncl = sh_ncl;
        const double pivfloor = __DBL_EPSILON__ * tnorm;
        for (int cb = 0; cb < ncl; cb += NT) {
            const int cl = cb + tid;
            if (tid < NT && cl < ncl) {
                double *u1 = lu + tid, *u2 = u1 + c * NT, *u3 = u2 + c * NT, *rr = u3 + c * NT;
                for (int g = cl_start[cl]; g < cl_start[cl + 1]; ++g) {
                    const double lmb = lam[g];
                    double *z = Z + g;                 // column g, stride kk
                    int attempt = 0;
                    for (int i = 0; i < c; ++i) z[i * kk] = start_value(i, g, attempt);
                    for (int it = 0; it < 2; ++it) {
                        // LU with partial pivoting of T - lmb I, applied to z.
                        double p0 = d[0] - lmb, p1 = c > 1 ? e[0] : 0.0, r = z[0];
                        for (int i = 0; i + 1 < c; ++i) {
                            const double sv = e[i], dd = d[i + 1] - lmb;
                            const double ee = (i + 2 < c) ? e[i + 1] : 0.0;
                            const double zn = z[(i + 1) * kk];
                            if (fabs(sv) > fabs(p0)) {       // swap rows i and i+1
                                const double mlt = p0 / sv;
                                u1[i * NT] = sv; u2[i * NT] = dd; u3[i * NT] = ee; rr[i * NT] = zn;
                                const double np0 = p1 - mlt * dd;
                                p1 = -mlt * ee;
                                r = r - mlt * zn;
                                p0 = np0;
                            } else {
                                double piv = p0;
                                if (fabs(piv) < pivfloor) piv = piv < 0.0 ? -pivfloor : pivfloor;
                                const double mlt = sv / piv;
                                u1[i * NT] = piv; u2[i * NT] = p1; u3[i * NT] = 0.0; rr[i * NT] = r;
                                p0 = dd - mlt * p1;
                                p1 = ee;
                                r = zn - mlt * r;
                            }
                        }
                        if (fabs(p0) < pivfloor) p0 = p0 < 0.0 ? -pivfloor : pivfloor;
                        double y2 = 0.0, y1 = r / p0;
                        z[(c - 1) * kk] = y1;
                        for (int i = c - 2; i >= 0; --i) {
                            const double y = (rr[i * NT] - u2[i * NT] * y1 - u3[i * NT] * y2) / u1[i * NT];
                            z[i * kk] = y;
                            y2 = y1;
                            y1 = y;
                        }
                        // Gram-Schmidt against earlier members of the cluster, normalise
                        for (int h = cl_start[cl]; h < g; ++h) {
                            const double *zh = Z + h;
                            double sd = 0.0;
                            for (int i = 0; i < c; ++i) sd = fma(zh[i * kk], z[i * kk], sd);
                            for (int i = 0; i < c; ++i) z[i * kk] -= sd * zh[i * kk];
                        }
                        double nrm = 0.0;
                        for (int i = 0; i < c; ++i) nrm = fma(z[i * kk], z[i * kk], nrm);
                        if (!(nrm > 0.0) || !isfinite(nrm)) {
                            ++attempt;               // restart from another vector
                            for (int i = 0; i < c; ++i) z[i * kk] = start_value(i, g, attempt);
                            continue;
                        }
                        const double inv = 1.0 / sqrt(nrm);
                        for (int i = 0; i < c; ++i) z[i * kk] *= inv;
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- 5. back-transformation x = H_0 H_1 ... H_{c-3} z, columns in registers ----
    {
        constexpr int CPW = kMaxK / kWaves;        // columns per wave, at most
        double z0[CPW], z1[CPW];
        const int ncol = (kk - wave + kWaves - 1) / kWaves;
#pragma unroll
        for (int u = 0; u < CPW; ++u) {
            const int g = wave + u * kWaves;
            z0[u] = (u < ncol && lane < c) ? Z[lane * kk + g] : 0.0;
            z1[u] = (u < ncol && lane + 64 < c) ? Z[(lane + 64) * kk + g] : 0.0;
        }
        if (ncol > 0) {
            for (int j = c - 3; j >= 0; --j) {
                const double t = tau[j];
                if (t == 0.0) continue;
                const int i0 = lane - (j + 1), i1 = lane + 64 - (j + 1);   // index into v_j
                const double *vj = A + hoff(j);
                const double v0 = (i0 >= 0 && lane < c) ? vj[i0] : 0.0;
                const double v1 = (i1 >= 0 && lane + 64 < c) ? vj[i1] : 0.0;
                double sv[CPW];
#pragma unroll
                for (int u = 0; u < CPW; ++u) sv[u] = fma(v0, z0[u], v1 * z1[u]);
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
                    for (int u = 0; u < CPW; ++u)
                        if (u < ncol) sv[u] += __shfl_xor(sv[u], off, 64);
#pragma unroll
                for (int u = 0; u < CPW; ++u) {
                    z0[u] -= t * sv[u] * v0;
                    z1[u] -= t * sv[u] * v1;
                }
            }
        }
        __syncthreads();                           // every wave has read its columns
#pragma unroll
        for (int u = 0; u < CPW; ++u) {
            const int g = wave + u * kWaves;
            if (u < ncol) {
                if (lane < c) Z[lane * kk + g] = z0[u];
                if (lane + 64 < c) Z[(lane + 64) * kk + g] = z1[u];
            }
        }
    }
    __syncthreads();

    // ---- 6. classical Gram-Schmidt, twice, on Z in LDS --------------------------------
    {
        double *dots = Z + c * kk;                 // kk (the solver arrays are free)
        for (int g = 0; g < kk; ++g) {
            int attempt = 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int h = wave; h < g; h += kWaves) {
                    double sd = 0.0;
                    for (int i = lane; i < c; i += 64) sd = fma(Z[i * kk + h], Z[i * kk + g], sd);
                    sd = wave_sum(sd);
                    if (lane == 0) dots[h] = sd;
                }
                __syncthreads();
                for (int i = tid; i < c; i += NTH) {
                    double v = Z[i * kk + g];
                    for (int h = 0; h < g; ++h) v -= dots[h] * Z[i * kk + h];
                    Z[i * kk + g] = v;
                }
                __syncthreads();
                double sn = 0.0;
                for (int i = lane; i < c; i += 64) sn = fma(Z[i * kk + g], Z[i * kk + g], sn);
                const double nrm2 = wave_sum(sn);  // every wave computes the same norm
                __syncthreads();
                if (pass == 1 && nrm2 < 0.25 && attempt < c) {
                    // collapsed inside a degenerate eigenspace: try the next unit vector
                    for (int i = tid; i < c; i += NTH)
                        Z[i * kk + g] = (i == (g + attempt) % c) ? 1.0 : 0.0;
                    ++attempt;
                    pass = -1;
                    __syncthreads();
                    continue;
                }
                const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
                for (int i = tid; i < c; i += NTH) Z[i * kk + g] *= inv;
                __syncthreads();
            }
        }
        for (int q = tid; q < c * kk; q += NTH) out[q] = Z[q];
    }
}

template <int NMAX>
hipError_t run_eig_tri(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                       const double *const *msrc, double *Vk, hipStream_t stream)
{
    const size_t lds = TriLayout<NMAX>::bytes();
    static size_t cur = 0;
    hipError_t e = ensure_lds((const void *)eig_tri_kernel<NMAX>, lds, cur);
    if (e != hipSuccess) return e;
    eig_tri_kernel<NMAX><<<nprob, NTH, lds, stream>>>(c, k, probs, gsrc, msrc, Vk);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eig_tri(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                          const double *const *msrc, double *Vk, hipStream_t stream)
{
    if (nprob <= 0) return hipSuccess;
    if (c > kMaxC) return hipErrorInvalidValue;
    timing_begin("eig", stream);
    hipError_t e;
    if (c <= 32) e = run_eig_tri<32>(c, k, probs, nprob, gsrc, msrc, Vk, stream);
    else if (c <= 64) e = run_eig_tri<64>(c, k, probs, nprob, gsrc, msrc, Vk, stream);
    else e = run_eig_tri<128>(c, k, probs, nprob, gsrc, msrc, Vk, stream);
    timing_end("eig", stream);
    return e;
}

}  // namespace zs
