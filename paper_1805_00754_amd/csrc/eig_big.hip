// Leading eigenvectors of a symmetric positive semi-definite c x c Gram matrix
// for 128 < c <= 1024, one work-group per matrix (512 threads up to c = 256,
// 1024 above), with the matrix in a global scratch slot and the vectors of
// each step in LDS.  Same method as the solver for c <= 128
// (eig_tri.hip), whose matrix fits in registers:
//
//   1. W <- the problem's Gram terms (tree nodes / block chunk Grams, then the
//      Grams of its Partial-SVD rows), in a fixed order.
//   2. Householder tridiagonalisation Q^T W Q = T in panels of NB steps
//      (blocked, below): the reflector of row j is formed in LDS and saved
//      over the dead part of row j; within a panel the trailing block is
//      only read (one matrix-vector product per step), and after the panel
//      it takes the panel's rank-2NB update on the FP64 matrix cores.
//   3. The kk largest eigenvalues of T by multisection on Sturm counts.
//   4. Eigenvectors of T by inverse iteration (tridiagonal LU with partial
//      pivoting, two solves, one thread per cluster of eigenvalues closer
//      than 1e-9 ||T||, Gram-Schmidt inside a cluster), arrays in scratch.
//   5. Back-transformation x = H_0 ... H_{c-3} z, several columns per wave
//      pass sharing each reflector's load.
//   6. Two passes of classical Gram-Schmidt (a collapsed vector is replaced
//      by the next unit vector, which only happens in a degenerate
//      eigenspace).
// Scratch per problem: c^2 + 5 c kk doubles (eig_big_scratch_doubles).
#include "zs_internal.h"
#include "wave.h"

namespace zs {
namespace {

constexpr int kBigMax = 1024;             // largest c
constexpr int kWU = 8;                    // matrix entries per thread in flight in phase 1

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the work-group; red holds kWaves doubles.  All threads call it.
template <int kWaves>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    v = wave_sum64(v);
    __syncthreads();                      // red is free
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += red[w];
    return s;
}

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

// VPL: vector entries per lane in phase 5 (c <= 64 VPL); NTH threads; CMAX:
// the largest c of the instantiation (sizes the LDS vectors); NB: steps per
// panel of the tridiagonal reduction; LCL: the panel's reflector columns in
// LDS (else in the problem's global scratch).
template <int VPL, int NTH, int CMAX, int NB, bool LCL>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4))) void eig_big_kernel(int c, int k, const Prob *__restrict__ probs,
                                                      const double *const *__restrict__ gsrc,
                                                      const double *const *__restrict__ msrc,
                                                      double *__restrict__ scratch,
                                                      double *__restrict__ Vk)
{
    constexpr int kWaves = NTH / 64;
    __shared__ double d[CMAX], e[CMAX], e2[CMAX], tau[CMAX];
    __shared__ double vbuf[CMAX], wbuf[CMAX];   // v and p / w of a step
    __shared__ double colb[CMAX];         // the next step's panel-start column
    __shared__ double rowb[CMAX];         // the next row to reduce, from its diagonal on
    __shared__ double xs[NTH];
    __shared__ int cs[NTH];
    __shared__ double lam[kMaxK], glo[kMaxK], ghi[kMaxK], red[kWaves];
    __shared__ int cl_start[kMaxK + 1];
    __shared__ double sh_a, sh_b, sh_tnorm, sh_pivmin;
    __shared__ int sh_ncl, sh_done;

    const Prob P = probs[blockIdx.x];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int kk = P.kk;
    double *W = scratch + (int64_t)blockIdx.x * ((int64_t)c * c + 5 * (int64_t)c * kMaxK);
    double *Z = W + (int64_t)c * c;                  // c x kk, row-major
    double *LU = Z + (int64_t)c * kMaxK;            // 4 arrays of c per solver thread
    double *out = Vk + (int64_t)blockIdx.x * c * kMaxK;

    // ---- 1. W (its lower triangle, the only part phase 2 reads) ------------------
    //      Each thread sums kWU entries at a time (independent loads in flight),
    //      each entry in the fixed term order.  Entries run over the packed
    //      lower triangle, row by row: q = i (i + 1) / 2 + l, l <= i.
    const int64_t cl = (int64_t)c * (c + 1) / 2;
    for (int64_t q0 = tid; q0 < cl; q0 += (int64_t)NTH * kWU) {
        double s[kWU];
        int64_t at[kWU];
#pragma unroll
        for (int x = 0; x < kWU; ++x) {
            s[x] = 0.0;
            const int64_t q = min(q0 + (int64_t)x * NTH, cl - 1);
            int64_t i = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
            while (i * (i + 1) / 2 > q) --i;
            while ((i + 1) * (i + 2) / 2 <= q) ++i;
            at[x] = i * c + (q - i * (i + 1) / 2);
        }
        for (int g = 0; g < P.ng; ++g) {
            const double *src = gsrc[P.g0 + g];
#pragma unroll
            for (int x = 0; x < kWU; ++x) s[x] += src[at[x]];
        }
#pragma unroll
        for (int x = 0; x < kWU; ++x)
            if (q0 + (int64_t)x * NTH < cl) W[at[x]] = s[x];
    }
    __syncthreads();
    // Grams of the Partial-SVD rows: W += R^T R, R k x c.  Each thread owns
    // 4 x 8 tiles of W (12 loads feed 32 FMAs per row of R); every entry is
    // still W(i, j) followed by the FMAs over the rows of R in order.
    {
        constexpr int TI = 4, TJ = 8;
        const int nti = (c + TI - 1) / TI, ntj = (c + TJ - 1) / TJ;
        for (int m = 0; m < P.nm; ++m) {
            const double *R = msrc[P.m0 + m];                   // k x c rows
            for (int tt = tid; tt < nti * ntj; tt += NTH) {
                const int i0 = (tt / ntj) * TI, j0 = (tt % ntj) * TJ;
                if (j0 > i0 + TI - 1) continue;           // no entry on or below the diagonal
                double acc[TI][TJ];
#pragma unroll
                for (int a = 0; a < TI; ++a)
#pragma unroll
                    for (int b = 0; b < TJ; ++b)
                        acc[a][b] = (i0 + a < c && j0 + b < c) ? W[(int64_t)(i0 + a) * c + j0 + b] : 0.0;
                for (int r = 0; r < k; ++r) {
                    const double *Rr = R + (int64_t)r * c;
                    double ri[TI], rj[TJ];
#pragma unroll
                    for (int a = 0; a < TI; ++a) ri[a] = Rr[min(i0 + a, c - 1)];
#pragma unroll
                    for (int b = 0; b < TJ; ++b) rj[b] = Rr[min(j0 + b, c - 1)];
#pragma unroll
                    for (int a = 0; a < TI; ++a)
#pragma unroll
                        for (int b = 0; b < TJ; ++b) acc[a][b] = fma(ri[a], rj[b], acc[a][b]);
                }
#pragma unroll
                for (int a = 0; a < TI; ++a)
#pragma unroll
                    for (int b = 0; b < TJ; ++b)
                        if (i0 + a < c && j0 + b < c) W[(int64_t)(i0 + a) * c + j0 + b] = acc[a][b];
            }
            __syncthreads();
        }
    }

    // ---- 2. tridiagonalisation, blocked ------------------------------------------
    // Panels of NB Householder steps (the blocked reduction of Golub & Van
    // Loan 8.3 / LAPACK's latrd).  Within a panel the trailing block of W is
    // not updated: step j works with A_eff = W - V Wp^T - Wp V^T, where the
    // columns of V and Wp are the panel's reflectors v and w so far, kept
    // column-major in Lc (2 NB x c: V then Wp, absolute row index, zero
    // outside (j, c)).  Only the lower triangle of the trailing block is
    // kept (W is symmetric); the upper part of row j is free for v_j.
    // Step j
    //   (1) forms row j of A_eff (panel-start column j minus the corrections),
    //   (2) derives the reflector (tau, e, d of j; v over the dead part of row j),
    //   (3) q = W v over the lower triangle of the trailing block (read only)
    //       and the 2t dots x = Wp^T v, y = V^T v,
    //   (4) p = tau (q - V x - Wp y), w = p - (tau/2)(p.v) v, appended to Lc.
    // After the panel the lower triangle of the trailing block takes the
    // whole rank-2NB update W -= [V Wp] [Wp V]^T on the FP64 matrix cores.
    // Each step reads half the trailing block once (the unblocked form read
    // and wrote all of it), and the panel update reads and writes half of
    // it once per NB steps.
    constexpr int RU = 4;                           // rows per wave in flight (3)
    constexpr int HM = CMAX / 64;                   // 64-column chunks of a row, at most
    static_assert((NB & (NB - 1)) == 0 && NB >= 2, "NB a power of two");
    __shared__ double lcs[LCL ? 2 * NB * CMAX : 1];
    __shared__ double gsh[LCL ? 1 : kMaxK * kMaxK];   // phase 6 (lcs serves when LCL)
    double *Lc = LCL ? lcs : Z;                     // 2 NB x c (Z is free until phase 4)
    double *vv = vbuf;                              // v of the step, local index u = i - j - 1
    double *qw = wbuf;                              // q, then p and w (local index)
    double *Pw = Z + (LCL ? 0 : (int64_t)2 * NB * c);   // kWaves x c column sums of step (3)
    double *xy = xs;                                // the 2t correction dots
    // Reflector of row jr (the row of A_eff in rowb, from its diagonal on):
    // tau, e, d of jr and v (length c - jr - 1, v(0) = 1) into vdst and over
    // the dead part of row jr in W.
    auto make_reflector = [&](int jr, double *vdst) {
        const int n = c - jr - 1;
        double *rowj = W + (int64_t)jr * c;
        double part = 0.0;
        for (int i = tid + 1; i < n; i += NTH) part = fma(rowb[1 + i], rowb[1 + i], part);
        const double s = block_sum<kWaves>(part, red);
        const double alpha = rowb[1];
        double t = 0.0, beta = alpha, scal = 0.0;
        if (s > 0.0) {
            const double mu = sqrt(alpha * alpha + s);
            beta = alpha <= 0.0 ? mu : -mu;
            t = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        if (tid == 0) {
            tau[jr] = t;
            e[jr] = beta;
            d[jr] = rowb[0];
        }
        for (int i = tid; i < n; i += NTH) vdst[i] = (i == 0) ? 1.0 : rowb[1 + i] * scal;
        __syncthreads();
        // v_jr replaces the dead entries of row jr (read back in phase 5)
        for (int i = tid; i < n; i += NTH) rowj[jr + 1 + i] = vdst[i];
    };
    typedef double v4d __attribute__((ext_vector_type(4)));
    for (int j0 = 0; j0 + 2 < c; j0 += NB) {
        const int nbp = min(NB, c - 2 - j0);       // steps of this panel
        // columns of an incomplete panel stay zero in the update
        for (int q = tid; q < (NB - nbp) * c; q += NTH) {
            const int t = nbp + q / c, i = q % c;
            Lc[(int64_t)t * c + i] = 0.0;
            Lc[(int64_t)(NB + t) * c + i] = 0.0;
        }
        for (int t = 0; t < nbp; ++t) {
            const int j = j0 + t;
            const int n = c - j - 1;               // trailing size
            // (1) row j of A_eff, columns j .. c-1, from the panel-start column j
            // (lower triangle: read at the panel's first step, else saved by
            // the previous step's product)
            for (int k = j + tid; k < c; k += NTH) {
                double r = t == 0 ? W[(int64_t)k * c + j] : colb[k];
                for (int s2 = 0; s2 < t; ++s2)
                    r -= Lc[(int64_t)s2 * c + j] * Lc[(int64_t)(NB + s2) * c + k] +
                         Lc[(int64_t)(NB + s2) * c + j] * Lc[(int64_t)s2 * c + k];
                rowb[k - j] = r;
            }
            __syncthreads();
            // (2) the reflector of row j
            make_reflector(j, vv);
            __syncthreads();                       // v is visible; row j of W holds v
            const double tj = tau[j];
            // (3) q = W v over rows and columns (j, c) of the panel-start block,
            // from its lower triangle: element (i, l), l <= i, adds W(i, l) v_l
            // to q_i (row sum, one wave sum per row) and, for l < i, W(i, l) v_i
            // to q_l (column sums kept per lane over the wave's rows, then
            // added across the waves in a fixed order in step (4)).
            const double *Wt = W + (int64_t)(j + 1) * c + (j + 1);
            double colacc[HM];
#pragma unroll
            for (int h = 0; h < HM; ++h) colacc[h] = 0.0;
            for (int q0 = wave * RU; q0 < n; q0 += kWaves * RU) {
                double acc[RU], vi[RU];
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    acc[u] = 0.0;
                    vi[u] = q0 + u < n ? vv[q0 + u] : 0.0;
                }
                const int hl = min(q0 + RU, n) - 1;        // the group's last (longest) row
#pragma unroll
                for (int h = 0; h < HM; ++h) {
                    if (64 * h <= hl) {
                        const int l = 64 * h + lane;
                        const double vl = l < n ? vv[l] : 0.0;
                        double x[RU];
#pragma unroll
                        for (int u = 0; u < RU; ++u)
                            x[u] = (l <= q0 + u && q0 + u < n) ? Wt[(int64_t)(q0 + u) * c + l] : 0.0;
#pragma unroll
                        for (int u = 0; u < RU; ++u) {
                            acc[u] = fma(x[u], vl, acc[u]);
                            colacc[h] = fma(l < q0 + u ? x[u] : 0.0, vi[u], colacc[h]);
                        }
                        if (h == 0 && lane == 0) {         // column j + 1 for the next step
#pragma unroll
                            for (int u = 0; u < RU; ++u)
                                if (q0 + u < n) colb[j + 1 + q0 + u] = x[u];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const double sdot = wave_sum64(acc[u]);
                    if (lane == 0 && q0 + u < n) qw[q0 + u] = sdot;
                }
            }
#pragma unroll
            for (int h = 0; h < HM; ++h) {
                const int l = 64 * h + lane;
                if (l < n) Pw[(int64_t)wave * c + l] = colacc[h];
            }
            // the 2t dots: x_s = Wp(:, s)^T v (dd < t), y_s = V(:, s)^T v
            // (t <= dd < 2t), half a wave per dot
            for (int dd = tid / 32; dd < 2 * t; dd += NTH / 32) {
                const double *col = dd < t ? Lc + (int64_t)(NB + dd) * c : Lc + (int64_t)(dd - t) * c;
                double acc = 0.0;
                for (int u = tid % 32; u < n; u += 32) acc = fma(col[j + 1 + u], vv[u], acc);
                acc = row16_sum(acc);
                // the two halves' sums, read with wave-uniform lanes
                const double s0 = readlane_d(acc, 0) + readlane_d(acc, 16);
                const double s1 = readlane_d(acc, 32) + readlane_d(acc, 48);
                if ((tid % 32) == 0) xy[dd] = lane < 32 ? s0 : s1;
            }
            // both halves of a wave must take part in the lane reads above
            __syncthreads();
            // (4) p = tau (q - V x - Wp y), then K = (tau/2) p.v and w = p - K v
            double pk = 0.0;
            for (int u = tid; u < n; u += NTH) {
                const int i = j + 1 + u;
                double pv = qw[u];
                for (int w2 = 0; w2 < kWaves; ++w2) pv += Pw[(int64_t)w2 * c + u];
                for (int s2 = 0; s2 < t; ++s2)
                    pv -= Lc[(int64_t)s2 * c + i] * xy[s2] + Lc[(int64_t)(NB + s2) * c + i] * xy[t + s2];
                pv *= tj;
                qw[u] = pv;
                pk = fma(pv, vv[u], pk);
            }
            const double K = 0.5 * tj * block_sum<kWaves>(pk, red);
            for (int i = tid; i < c; i += NTH) {
                const int u = i - j - 1;
                const double vi = u >= 0 ? vv[u] : 0.0;
                const double wi = u >= 0 ? qw[u] - K * vi : 0.0;
                Lc[(int64_t)t * c + i] = vi;
                Lc[(int64_t)(NB + t) * c + i] = wi;
            }
            __syncthreads();                       // the panel's columns are complete
        }
        // (5) W(m0:c, m0:c) -= [V Wp] [Wp V]^T on its lower triangle, on the
        // FP64 16x16x4 shape: a wave takes a strip of 16 rows (its A
        // fragments A(i, s) = Lc(s, i) in lane i + 16 s stay in registers)
        // and walks its 16 x 16 blocks up to the diagonal;
        // B(s, jj) = Lc(s ^ NB, jj) in lane jj + 16 s, D(i, jj) in register
        // i / 4 of lane jj + 16 (i mod 4).
        {
            const int m0 = j0 + nbp;
            const int nrs = (c - m0 + 15) / 16;
            constexpr int QS = 2 * NB / 4;             // MFMA steps over the 2 NB columns
            for (int r = wave; r < nrs; r += kWaves) {
                const int i0 = m0 + 16 * r;
                const int ia = i0 + lane % 16;
                double af[QS];
#pragma unroll
                for (int q = 0; q < QS; ++q) {
                    const int sa = 4 * q + lane / 16;
                    if constexpr (LCL) {
                        af[q] = ia < c ? Lc[(int64_t)sa * c + ia] : 0.0;
                    } else {
                        const double ar = Lc[(int64_t)sa * c + min(ia, c - 1)];
                        af[q] = ia < c ? ar : 0.0;
                    }
                }
                const int nblk = r + 1;                // blocks from column m0 to the diagonal
                for (int b0 = 0; b0 < nblk; ++b0) {
                    v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
                    const int kb = m0 + 16 * b0 + lane % 16, kc = min(kb, c - 1);
                    if constexpr (LCL) {
                        // panel columns in LDS: loads as needed
#pragma unroll
                        for (int q = 0; q < QS; ++q) {
                            const int sb = (4 * q + lane / 16) ^ NB;
                            const double bv = kb < c ? Lc[(int64_t)sb * c + kb] : 0.0;
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[q], bv, acc, 0, 0, 0);
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = i0 + 4 * v + lane / 16;
                            if (i < c && kb < c) W[(int64_t)i * c + kb] -= acc[v];
                        }
                    } else {
                        // panel columns and W from cache: every load issued
                        // (clamped) before the first use
                        double bv[QS], wv[4];
#pragma unroll
                        for (int q = 0; q < QS; ++q) {
                            const int sb = (4 * q + lane / 16) ^ NB;
                            const double br = Lc[(int64_t)sb * c + kc];
                            bv[q] = kb < c ? br : 0.0;
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            wv[v] = W[(int64_t)min(i0 + 4 * v + lane / 16, c - 1) * c + kc];
#pragma unroll
                        for (int q = 0; q < QS; ++q)
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[q], bv[q], acc, 0, 0, 0);
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = i0 + 4 * v + lane / 16;
                            if (i < c && kb < c) W[(int64_t)i * c + kb] = wv[v] - acc[v];
                        }
                    }
                }
            }
        }
        __syncthreads();                           // the trailing block is updated
    }
    if (tid == 0) {                                // the last 2 x 2 block
        d[c - 2] = W[(int64_t)(c - 2) * c + c - 2];
        e[c - 2] = W[(int64_t)(c - 1) * c + c - 2];
        rowb[0] = W[(int64_t)(c - 1) * c + c - 1];
    }
    __syncthreads();
    if (tid == 0) {
        d[c - 1] = rowb[0];                        // row c-1, kept by the last pass
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
    __syncthreads();                               // d, e complete
    for (int i = tid; i + 1 < c; i += NTH) e2[i] = e[i] * e[i];
    __syncthreads();
    const double tnorm = sh_tnorm, pivmin = sh_pivmin;
    if (tnorm == 0.0) {
        for (int q = tid; q < c * kk; q += NTH) out[q] = (q / kk == q % kk) ? 1.0 : 0.0;
        return;
    }

    // ---- 3. the kk largest eigenvalues: multisection on Sturm counts ---------------
    {
        const int G = min(NTH / kk, 64);
        const int grp = tid / G, mem = tid % G;
        const int m = c - 1 - grp;
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
    if (tid == 0) {
        int n = 0;
        cl_start[n++] = 0;
        for (int g = 1; g < kk; ++g)
            if (lam[g - 1] - lam[g] > 1e-9 * tnorm) cl_start[n++] = g;
        cl_start[n] = kk;
        sh_ncl = n;
    }
    __syncthreads();

    // ---- 4. inverse iteration: one thread per cluster ------------------------------
    {
        const int ncl = sh_ncl;
        const double pivfloor = __DBL_EPSILON__ * tnorm;
        if (tid < ncl) {
            const int cl = tid;
            double *u1 = LU + (int64_t)4 * c * tid, *u2 = u1 + c, *u3 = u2 + c, *rr = u3 + c;
            for (int g = cl_start[cl]; g < cl_start[cl + 1]; ++g) {
                const double lmb = lam[g];
                double *z = Z + g;                   // column g, stride kk
                int attempt = 0;
                for (int i = 0; i < c; ++i) z[(int64_t)i * kk] = start_value(i, g, attempt);
                for (int it = 0; it < 2; ++it) {
                    double p0 = d[0] - lmb, p1 = c > 1 ? e[0] : 0.0, r = z[0];
                    for (int i = 0; i + 1 < c; ++i) {
                        const double sv = e[i], dd = d[i + 1] - lmb;
                        const double ee = (i + 2 < c) ? e[i + 1] : 0.0;
                        const double zn = z[(int64_t)(i + 1) * kk];
                        if (fabs(sv) > fabs(p0)) {
                            const double mlt = p0 / sv;
                            u1[i] = sv; u2[i] = dd; u3[i] = ee; rr[i] = zn;
                            const double np0 = p1 - mlt * dd;
                            p1 = -mlt * ee;
                            r = r - mlt * zn;
                            p0 = np0;
                        } else {
                            double piv = p0;
                            if (fabs(piv) < pivfloor) piv = piv < 0.0 ? -pivfloor : pivfloor;
                            const double mlt = sv / piv;
                            u1[i] = piv; u2[i] = p1; u3[i] = 0.0; rr[i] = r;
                            p0 = dd - mlt * p1;
                            p1 = ee;
                            r = zn - mlt * r;
                        }
                    }
                    if (fabs(p0) < pivfloor) p0 = p0 < 0.0 ? -pivfloor : pivfloor;
                    double y2 = 0.0, y1 = r / p0;
                    z[(int64_t)(c - 1) * kk] = y1;
                    for (int i = c - 2; i >= 0; --i) {
                        const double y = (rr[i] - u2[i] * y1 - u3[i] * y2) / u1[i];
                        z[(int64_t)i * kk] = y;
                        y2 = y1;
                        y1 = y;
                    }
                    for (int h = cl_start[cl]; h < g; ++h) {
                        const double *zh = Z + h;
                        double sd = 0.0;
                        for (int i = 0; i < c; ++i) sd = fma(zh[(int64_t)i * kk], z[(int64_t)i * kk], sd);
                        for (int i = 0; i < c; ++i) z[(int64_t)i * kk] -= sd * zh[(int64_t)i * kk];
                    }
                    double nrm = 0.0;
                    for (int i = 0; i < c; ++i) nrm = fma(z[(int64_t)i * kk], z[(int64_t)i * kk], nrm);
                    if (!(nrm > 0.0) || !isfinite(nrm)) {
                        ++attempt;
                        for (int i = 0; i < c; ++i) z[(int64_t)i * kk] = start_value(i, g, attempt);
                        continue;
                    }
                    const double inv = 1.0 / sqrt(nrm);
                    for (int i = 0; i < c; ++i) z[(int64_t)i * kk] *= inv;
                }
            }
        }
        __threadfence_block();
        __syncthreads();
    }

    // ---- 5. back-transformation: CPP columns per wave pass -----------------------
    //      The columns of a pass share each reflector's load; up to c = 512 the
    //      next reflector is loaded while this one is applied (above, the
    //      registers are not there for it).
    {
        constexpr int CPP = VPL <= 4 ? 4 : 2;
        constexpr bool PRE = VPL <= 8;
        auto vload = [&](int j, double (&v)[VPL]) {
            const double *vj = W + (int64_t)max(j, 0) * c + max(j, 0) + 1;   // v_j(i') at vj[i']
#pragma unroll
            for (int u = 0; u < VPL; ++u) {
                const int i = lane + 64 * u;
                v[u] = (j >= 0 && i >= j + 1 && i < c) ? vj[i - j - 1] : 0.0;
            }
        };
        for (int g0 = wave * CPP; g0 < kk; g0 += kWaves * CPP) {
            double z[CPP][VPL];
#pragma unroll
            for (int h = 0; h < CPP; ++h)
#pragma unroll
                for (int u = 0; u < VPL; ++u) {
                    const int i = lane + 64 * u;
                    z[h][u] = (g0 + h < kk && i < c) ? Z[(int64_t)i * kk + g0 + h] : 0.0;
                }
            double vq[VPL], vn[PRE ? VPL : 1];
            if constexpr (PRE) vload(c - 3, vq);
            for (int j = c - 3; j >= 0; --j) {
                if constexpr (PRE) vload(j - 1, vn);
                else vload(j, vq);
                const double t = tau[j];
                if (t != 0.0) {
#pragma unroll
                    for (int h = 0; h < CPP; ++h) {
                        double s0 = 0.0;
#pragma unroll
                        for (int u = 0; u < VPL; ++u) s0 = fma(vq[u], z[h][u], s0);
                        s0 = t * wave_sum64(s0);
#pragma unroll
                        for (int u = 0; u < VPL; ++u) z[h][u] -= s0 * vq[u];
                    }
                }
                if constexpr (PRE)
#pragma unroll
                    for (int u = 0; u < VPL; ++u) vq[u] = vn[u];
            }
#pragma unroll
            for (int h = 0; h < CPP; ++h)
#pragma unroll
                for (int u = 0; u < VPL; ++u) {
                    const int i = lane + 64 * u;
                    if (g0 + h < kk && i < c) Z[(int64_t)i * kk + g0 + h] = z[h][u];
                }
        }
    }
    __syncthreads();

    // ---- 6. orthonormalisation: Cholesky QR, twice ----------------------------------
    //      G = Z^T Z (4 x 4 blocks of its upper triangle, P threads of one wave
    //      per block, summed by a fixed butterfly), G = R^T R by one wave,
    //      R^-1 by one wave (row a of R^-1 is lane a's), Z <- Z R^-1 one row
    //      per thread (16-column blocks from the last, in place).  Z R^-1 is
    //      the Gram-Schmidt basis of Z; a pivot below 1/4 (a column that
    //      collapses, only in a degenerate eigenspace) sends the vectors to
    //      classical Gram-Schmidt below instead.
    double *Gs = LCL ? lcs : gsh;                   // kk x kk: R above the diagonal, R^-1 below
    double *rdi = xs;                               // diagonal of R^-1
    bool chol_ok = true;
    for (int round = 0; round < 2 && chol_ok; ++round) {
        {
            const int nb4 = (kk + 3) / 4, nblk = nb4 * (nb4 + 1) / 2;
            int P = 64;
            while (P > 1 && P * nblk > NTH) P >>= 1;
            const int blk = tid / P, part = tid % P;
            double acc[4][4];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
            int ba = 0, bb = 0;
            if (blk < nblk) {
                int r = blk;
                while (r >= nb4 - ba) {
                    r -= nb4 - ba;
                    ++ba;
                }
                bb = ba + r;
                for (int i = part; i < c; i += P) {
                    const double *zr = Z + (int64_t)i * kk;
                    double za[4], zb[4];
#pragma unroll
                    for (int x = 0; x < 4; ++x) {
                        za[x] = 4 * ba + x < kk ? zr[4 * ba + x] : 0.0;
                        zb[x] = 4 * bb + x < kk ? zr[4 * bb + x] : 0.0;
                    }
#pragma unroll
                    for (int x = 0; x < 4; ++x)
#pragma unroll
                        for (int y = 0; y < 4; ++y) acc[x][y] = fma(za[x], zb[y], acc[x][y]);
                }
            }
            for (int off = P / 2; off >= 1; off >>= 1)
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] += __shfl_xor(acc[x][y], off, 64);
            if (blk < nblk && part == 0)
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) {
                        const int a = 4 * ba + x, b = 4 * bb + y;
                        if (a < kk && b < kk) Gs[a * kk + b] = acc[x][y];
                    }
        }
        __syncthreads();
        if (wave == 0) {
            // right-looking Cholesky on the upper triangle, lane l owns column l
            int good = 1;
            for (int jj = 0; jj < kk; ++jj) {
                const double djj = Gs[jj * kk + jj];
                good &= djj > 0.25;
                const double rjj = sqrt(fmax(djj, 0.25));
                const double rjl = (lane > jj && lane < kk) ? Gs[jj * kk + lane] / rjj : 0.0;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane == jj) Gs[jj * kk + jj] = rjj;
                if (lane > jj && lane < kk) Gs[jj * kk + lane] = rjl;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int lp = jj + 1; lp < kk; ++lp) {
                    const double r1 = Gs[jj * kk + lp];
                    if (lane >= lp && lane < kk) Gs[lp * kk + lane] -= r1 * rjl;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            // R^-1: lane a computes row a, left to right
            if (lane < kk) {
                const int a = lane;
                const double ra = 1.0 / Gs[a * kk + a];
                rdi[a] = ra;
                for (int b = a + 1; b < kk; ++b) {
                    double sum = ra * Gs[a * kk + b];
                    for (int p2 = a + 1; p2 < b; ++p2) sum = fma(Gs[p2 * kk + a], Gs[p2 * kk + b], sum);
                    Gs[b * kk + a] = -sum / Gs[b * kk + b];
                }
            }
            if (lane == 0) sh_done = good;
        }
        __syncthreads();
        chol_ok = sh_done != 0;
        if (!chol_ok) break;
        for (int i = tid; i < c; i += NTH) {
            double *zr = Z + (int64_t)i * kk;
            for (int b0 = ((kk - 1) / 16) * 16; b0 >= 0; b0 -= 16) {
                double acc[16];
#pragma unroll
                for (int y = 0; y < 16; ++y) acc[y] = 0.0;
                const int amax = min(b0 + 16, kk);
                for (int a = 0; a < amax; ++a) {
                    const double za = zr[a];
#pragma unroll
                    for (int y = 0; y < 16; ++y) {
                        const int b = b0 + y;
                        if (b < kk && a <= b) acc[y] = fma(za, a == b ? rdi[a] : Gs[b * kk + a], acc[y]);
                    }
                }
#pragma unroll
                for (int y = 0; y < 16; ++y)
                    if (b0 + y < kk) zr[b0 + y] = acc[y];
            }
        }
        __threadfence_block();
        __syncthreads();
    }
    // ---- 6b. classical Gram-Schmidt, twice (when Cholesky QR stopped) -----------------
    for (int g = 0; g < (chol_ok ? 0 : kk); ++g) {
        int attempt = 0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int h = wave; h < g; h += kWaves) {
                double sd = 0.0;
                for (int i = lane; i < c; i += 64) sd = fma(Z[(int64_t)i * kk + h], Z[(int64_t)i * kk + g], sd);
                sd = wave_sum(sd);
                if (lane == 0) xs[h] = sd;
            }
            __threadfence_block();
            __syncthreads();
            double sn = 0.0;
            for (int i = tid; i < c; i += NTH) {
                double v = Z[(int64_t)i * kk + g];
                for (int h = 0; h < g; ++h) v -= xs[h] * Z[(int64_t)i * kk + h];
                Z[(int64_t)i * kk + g] = v;
                sn = fma(v, v, sn);
            }
            const double nrm2 = block_sum<kWaves>(sn, red);
            if (pass == 1 && nrm2 < 0.25 && attempt < c) {
                for (int i = tid; i < c; i += NTH)
                    Z[(int64_t)i * kk + g] = (i == (g + attempt) % c) ? 1.0 : 0.0;
                ++attempt;
                pass = -1;
                __threadfence_block();
                __syncthreads();
                continue;
            }
            const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
            for (int i = tid; i < c; i += NTH) Z[(int64_t)i * kk + g] *= inv;
            __threadfence_block();
            __syncthreads();
        }
    }
    for (int q = tid; q < c * kk; q += NTH) out[q] = Z[q];
}

}  // namespace

size_t eig_big_scratch_doubles(int c) { return (size_t)c * c + 5 * (size_t)c * kMaxK; }

hipError_t launch_eig_big(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                          const double *const *msrc, double *scratch, double *Vk, hipStream_t stream)
{
    if (nprob <= 0) return hipSuccess;
    if (c > kBigMax) return hipErrorInvalidValue;
    timing_begin("eig", stream);
    // c <= 256: 512 threads and LDS sized for 256, so that two matrices share
    // a CU (the steps of one matrix are latency-bound at this size); the same
    // form for every launch, so a problem's bits do not depend on the batch
    if (c <= 256)
        eig_big_kernel<4, 512, 256, 8, true><<<nprob, 512, 0, stream>>>(c, k, probs, gsrc, msrc,
                                                                         scratch, Vk);
    else if (c <= 512)
        eig_big_kernel<8, 1024, 512, 16, false><<<nprob, 1024, 0, stream>>>(c, k, probs, gsrc, msrc,
                                                                            scratch, Vk);
    else
        eig_big_kernel<16, 1024, kBigMax, 16, false><<<nprob, 1024, 0, stream>>>(c, k, probs, gsrc,
                                                                                 msrc, scratch, Vk);
    hipError_t e = hipGetLastError();
    timing_end("eig", stream);
    return e;
}

}  // namespace zs
