// Small symmetric eigen-solves (n <= 64) and the kernels built on them:
//
//  * finalize: second stage of every rank-k SVD (V_k is overwritten by
//    V_k W).  With Y = X V_k (the data
//    projected on the first-stage eigenvectors), G_Y = Y^T Y is nearly
//    diagonal with scales sigma_j^2; two-sided Jacobi on it (Demmel-Veselic
//    stopping rule) gives singular values with high relative accuracy
//    (Rayleigh-Ritz on span V_k).  Outputs Sigma, V = V_k W (sign rule
//    applied) and F = W Sigma^-1, so that U = Y F.
//  * partial: Partial-SVD of a boundary block (Alg. 3, Eqs. (5)-(6)):
//    P = X U_(i) Sigma_(i),  P^T P = V~ Sigma~^2 V~^T, the block's stack rows
//    Sigma~ V~^T V_(i)^T, and T = Sigma_(i) V~ Sigma~^+ so that U' = X U_(i) T.
#include <climits>

#include "zs_internal.h"

namespace zs {
namespace {


__device__ __forceinline__ void rr_pair(int step, int pi, int N, int &p, int &q)
{
    const int m = N - 1;
    if (pi == 0) {
        p = 0;
        q = 1 + (step % m);
    } else {
        p = 1 + ((pi + step) % m);
        q = 1 + ((m - pi + step) % m);
    }
}

// Two-sided cyclic Jacobi, parallel round-robin ordering, on the symmetric
// n x n matrix G (row-major, leading dimension ld) accumulating W (ld, identity on
// entry).  A pair is rotated when |g_pq| > tol sqrt(g_pp g_qq), tol = n eps
// (the relative stopping rule of Demmel & Veselic).  As in the classical
// algorithm, the rotated 2 x 2 block is set exactly afterwards: g_pq = 0,
// g_pp - t g_pq, g_qq + t g_pq, so no rounding residue is left in the
// annihilated entry.  Diagonal entries at or below (n eps)^2 tr(G) are
// numerically zero and are not rotated.
// Returns the number of sweeps, or -1 if the cap was hit.  All threads of
// the block must call it; cs/sn/dp/dq need n/2 entries.
// Sweep cap of every Jacobi solve on this device (kMaxSweeps unless a test
// lowers it to force ZS_ENOCONV).
__device__ int d_sweep_cap = kMaxSweeps;

__device__ int sym_jacobi(double *G, double *W, int n, int ld, double *cs_sh, double *sn_sh,
                          double *dp_sh, double *dq_sh, int *flag_sh, double *tr_sh)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        double tr = 0.0;
        for (int i = 0; i < n; ++i) tr += fabs(G[i * ld + i]);
        *tr_sh = tr;
    }
    __syncthreads();
    const double tol = (double)n * __DBL_EPSILON__;
    const double floor = ((double)n * __DBL_EPSILON__) * ((double)n * __DBL_EPSILON__) * (*tr_sh);
    const int N = (n + 1) & ~1;
    const int np = N / 2;
    const int cap = d_sweep_cap;
    for (int sweep = 1; sweep <= cap; ++sweep) {
        if (tid == 0) *flag_sh = 0;
        __syncthreads();
        for (int step = 0; step < N - 1; ++step) {
            for (int pi = tid; pi < np; pi += kThreads) {
                int p, q;
                rr_pair(step, pi, N, p, q);
                double cs = 1.0, sn = 0.0, dp = 0.0, dq = 0.0;
                if (p < n && q < n) {
                    const double gpp = G[p * ld + p], gqq = G[q * ld + q];
                    const double gpq = G[p * ld + q];
                    if (gpq != 0.0 && fabs(gpp) > floor && fabs(gqq) > floor &&
                        fabs(gpq) > tol * sqrt(fabs(gpp)) * sqrt(fabs(gqq))) {
                        const double zeta = (gqq - gpp) / (2.0 * gpq);
                        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        cs = 1.0 / sqrt(1.0 + t * t);
                        sn = cs * t;
                        dp = gpp - t * gpq;
                        dq = gqq + t * gpq;
                        *flag_sh = 1;
                    }
                }
                cs_sh[pi] = cs;
                sn_sh[pi] = sn;
                dp_sh[pi] = dp;
                dq_sh[pi] = dq;
            }
            __syncthreads();
            // columns p, q of G and W: G <- G J, W <- W J
            for (int e = tid; e < np * n; e += kThreads) {
                const int pi = e / n, r = e % n;
                const double sn = sn_sh[pi];
                if (sn == 0.0) continue;
                const double cs = cs_sh[pi];
                int p, q;
                rr_pair(step, pi, N, p, q);
                double gp = G[r * ld + p], gq = G[r * ld + q];
                G[r * ld + p] = cs * gp - sn * gq;
                G[r * ld + q] = sn * gp + cs * gq;
                gp = W[r * ld + p];
                gq = W[r * ld + q];
                W[r * ld + p] = cs * gp - sn * gq;
                W[r * ld + q] = sn * gp + cs * gq;
            }
            __syncthreads();
            // rows p, q of G: G <- J^T G
            for (int e = tid; e < np * n; e += kThreads) {
                const int pi = e / n, r = e % n;
                const double sn = sn_sh[pi];
                if (sn == 0.0) continue;
                const double cs = cs_sh[pi];
                int p, q;
                rr_pair(step, pi, N, p, q);
                const double gp = G[p * ld + r], gq = G[q * ld + r];
                G[p * ld + r] = cs * gp - sn * gq;
                G[q * ld + r] = sn * gp + cs * gq;
            }
            __syncthreads();
            // the rotated 2 x 2 blocks, exactly
            for (int pi = tid; pi < np; pi += kThreads) {
                if (sn_sh[pi] == 0.0) continue;
                int p, q;
                rr_pair(step, pi, N, p, q);
                G[p * ld + p] = dp_sh[pi];
                G[q * ld + q] = dq_sh[pi];
                G[p * ld + q] = 0.0;
                G[q * ld + p] = 0.0;
            }
            __syncthreads();
        }
        const int f = *flag_sh;
        __syncthreads();
        if (!f) return sweep;
    }
    return -1;
}

constexpr int kFinRows = 64;   // rows of V_k staged at a time by finalize

// Energy threshold of Eq. (1): triplet j (of rank pos[j] in descending order)
// is kept when the squared singular values ranked above it, summed in that
// order, stay below xi times the total energy.  Off unless 0 < xi < 1.
__device__ __forceinline__ bool xi_keep(const double *sig, const int *inv, int p, double xi,
                                        double total)
{
    if (!(xi > 0.0 && xi < 1.0) || !(total > 0.0)) return true;
    double run = 0.0;
    for (int i = 0; i < p; ++i) run += sig[inv[i]] * sig[inv[i]];
    return run < xi * total;
}

// Deterministic sum of one value per thread of the work-group (fixed tree).
__device__ double block_sum(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = kThreads / 2; s >= 1; s /= 2) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kThreads) void finalize_kernel(int c, int k, const Prob *__restrict__ probs,
                                                            const double *__restrict__ GYpart,
                                                            double *__restrict__ Vk,
                                                            double *__restrict__ F,
                                                            double rank_tol, int kk_max,
                                                            const double *const *__restrict__ gsrc,
                                                            const double *const *__restrict__ msrc,
                                                            double xi, int *__restrict__ conv_flag)
{
    extern __shared__ __align__(16) double smem[];
    const int ld = kk_max + 1;                // leading dimension of the kk x kk matrices
    double *G = smem;                         // kk x kk
    double *W = G + kk_max * ld;              // kk x kk
    double *Rs = W + kk_max * ld;             // kFinRows x kk rows of V_k
    __shared__ double cs_sh[kMaxK / 2], sn_sh[kMaxK / 2], dp_sh[kMaxK / 2], dq_sh[kMaxK / 2];
    __shared__ double sig[kMaxK], flip[kMaxK];
    __shared__ int pos[kMaxK], inv[kMaxK], keep[kMaxK];
    __shared__ int flag_sh;
    __shared__ double tr_sh;
    __shared__ double red[kThreads];
    __shared__ int pidx_sh[kThreads];

    const Prob P = probs[blockIdx.x];
    const int kk = P.kk;
    const int tid = threadIdx.x;
    // total energy of the matrix whose SVD this is (the denominator of
    // Eq. (1)): the trace of its c x c Gram, term by term
    double total = 0.0;
    if (xi > 0.0 && xi < 1.0) {
        double part = 0.0;
        for (int g = 0; g < P.ng; ++g) {
            const double *Gs = gsrc[P.g0 + g];
            for (int a = tid; a < c; a += kThreads) part += Gs[(int64_t)a * c + a];
        }
        for (int m = 0; m < P.nm; ++m) {
            const double *R = msrc[P.m0 + m];
            for (int e = tid; e < k * c; e += kThreads) part += R[e] * R[e];
        }
        total = block_sum(part, red);
    }
    for (int e = tid; e < kk * kk; e += kThreads) {
        const int a = e / kk, b = e % kk;
        double s = 0.0;
        for (int sl = 0; sl < P.ny; ++sl) s += GYpart[(int64_t)(P.y0 + sl) * kSlotK + e];
        G[a * ld + b] = s;
        W[a * ld + b] = (a == b) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int sweeps = sym_jacobi(G, W, kk, ld, cs_sh, sn_sh, dp_sh, dq_sh, &flag_sh, &tr_sh);
    if (sweeps < 0 && tid == 0) atomicOr(conv_flag, 1);

    for (int j = tid; j < kk; j += kThreads) sig[j] = sqrt(fmax(G[j * ld + j], 0.0));
    __syncthreads();
    double smax = 0.0;
    for (int j = 0; j < kk; ++j) smax = fmax(smax, sig[j]);
    for (int j = tid; j < kk; j += kThreads) {
        int p = 0;
        for (int i = 0; i < kk; ++i) p += (sig[i] > sig[j]) || (sig[i] == sig[j] && i < j);
        pos[j] = p;
        inv[p] = j;
    }
    __syncthreads();
    for (int j = tid; j < kk; j += kThreads)
        keep[j] = (sig[j] > rank_tol * smax) && (sig[j] > 0.0) && xi_keep(sig, inv, pos[j], xi, total);
    // Vn = V_k W, in place over V_k (no longer needed), kFinRows rows at a time
    double *Vn = Vk + (int64_t)blockIdx.x * c * kMaxK;
    for (int a0 = 0; a0 < c; a0 += kFinRows) {
        const int nr = min(kFinRows, c - a0);
        __syncthreads();
        for (int e = tid; e < nr * kk; e += kThreads) Rs[e] = Vn[(int64_t)a0 * kk + e];
        __syncthreads();
        for (int e = tid; e < nr * kk; e += kThreads) {
            const int a = e / kk, j = e % kk;
            double s = 0.0;
            for (int l = 0; l < kk; ++l) s = fma(Rs[a * kk + l], W[l * ld + j], s);
            Vn[(int64_t)a0 * kk + e] = s;
        }
    }
    __threadfence_block();
    __syncthreads();
    // sign rule: largest |v| entry (lowest index on ties) made positive.
    // nsub (at most 16) threads per column each scan the rows a = sub mod
    // nsub in order (the first of equal maxima kept), then one thread per
    // column combines the partial maxima, equal values going to the lower
    // row: the entry a single scan over all rows would pick.
    {
        const int nsub = kk > 0 ? min(kThreads / kk, 16) : 1;
        if (tid < nsub * kk) {
            const int j = tid % kk, sub = tid / kk;
            int am = INT_MAX;
            double vm = -1.0;
            for (int a = sub; a < c; a += nsub) {
                const double v = fabs(Vn[(int64_t)a * kk + j]);
                if (v > vm) { vm = v; am = a; }
            }
            red[tid] = vm;
            pidx_sh[tid] = am;
        }
        __syncthreads();
        for (int j = tid; j < kk; j += kThreads) {
            int am = INT_MAX;
            double vm = -1.0;
            for (int sub = 0; sub < nsub; ++sub) {
                const double v = red[sub * kk + j];
                const int a = pidx_sh[sub * kk + j];
                if (v > vm || (v == vm && a < am)) { vm = v; am = a; }
            }
            if (am == INT_MAX) am = 0;        // no entry above -1 (all NaN)
            flip[j] = Vn[(int64_t)am * kk + j] < 0.0 ? -1.0 : 1.0;
        }
    }
    __syncthreads();
    for (int e = tid; e < c * kk; e += kThreads) {
        const int a = e / kk, pp = e % kk;
        const int j = inv[pp];
        const double v = keep[j] ? flip[j] * Vn[(int64_t)a * kk + j] : 0.0;
        if (P.v_f32)
            static_cast<float *>(P.v_dst)[a * P.v_rs + pp * P.v_cs] = (float)v;
        else
            static_cast<double *>(P.v_dst)[a * P.v_rs + pp * P.v_cs] = v;
    }
    double *Fp = F + (int64_t)blockIdx.x * kSlotK;
    for (int e = tid; e < kk * kk; e += kThreads) {
        const int l = e / kk, pp = e % kk;
        const int j = inv[pp];
        Fp[l * kk + pp] = keep[j] ? flip[j] * W[l * ld + j] / sig[j] : 0.0;
    }
    for (int pp = tid; pp < kk; pp += kThreads) {
        const int j = inv[pp];
        P.s_dst[pp] = keep[j] ? sig[j] : 0.0;
    }
    if (tid == 0) {
        int n = 0;
        for (int j = 0; j < kk; ++j) n += keep[j];
        *P.k_dst = n;
    }
}

// Rows of P staged in LDS at a time: 16, or 8 above k = 32 so that two
// blocks share a CU's LDS at k = 64.  The Gram sums run over the rows in
// order either way.
__host__ __device__ inline int partial_rows(int k) { return k > 32 ? 8 : 16; }

// From k = 17 on the Gram sums run over 2 x 2 tiles on or below the
// diagonal, TPT tiles per thread (one up to k = 44): four loads from LDS feed
// four FMAs, where one entry per thread takes two loads per FMA.  Up to
// k = 16 (TPT = 0) each thread sums one entry, which keeps more threads busy
// when the loads are few.  Either way every entry is summed by one thread
// over the rows in order, so the two forms give the same bits.  With at most
// one tile per thread the kernel is held to 64 registers, so that eight
// blocks (32 waves) share a CU and a batch's boundary blocks run in one round.
template <int TPT> struct PartialOcc { static constexpr int waves = TPT <= 1 ? 8 : 1; };
constexpr int kPartialTileK = 17;
static_assert((kPartialTileK - 1) * (kPartialTileK - 1) <= kThreads,
              "one Gram entry per thread below the tile threshold");

template <typename TU, int TPT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(PartialOcc<TPT>::waves)))
void partial_kernel(StoreView st,
                                                           const Piece *__restrict__ pieces,
                                                           const int32_t *__restrict__ pidx,
                                                           double *__restrict__ Mp,
                                                           double *__restrict__ T, double rank_tol,
                                                           double xi, int *__restrict__ conv_flag)
{
    extern __shared__ __align__(16) double smem[];
    const int k = st.k;
    const int RB = partial_rows(k);
    const int ld = k + 1;                     // leading dimension of the k x k matrices
    double *G = smem;                         // k x k (G_P, then G_Y)
    double *W1 = G + k * ld;                  // eigenvectors: first stage, then V~
    double *Us = W1 + k * ld;                 // RB x k staged rows of P = X U Sigma
    double *Ys = Us + RB * k;                 // RB x k rows of Y = P W1
    __shared__ double cs_sh[kMaxK / 2], sn_sh[kMaxK / 2], dp_sh[kMaxK / 2], dq_sh[kMaxK / 2];
    __shared__ double sig[kMaxK], sblk[kMaxK];
    __shared__ int pinv[kMaxK], pkeep[kMaxK];
    __shared__ int flag_sh;
    __shared__ double tr_sh;

    const Piece pc = pieces[pidx[blockIdx.x]];
    const int c = (int)st.c;
    const int tid = threadIdx.x;
    const TU *Ub = static_cast<const TU *>(st.U) + (pc.blk * st.b + pc.r0) * k;
    const int m = pc.r1 - pc.r0;
    for (int j = tid; j < k; j += kThreads) sblk[j] = st.S[pc.blk * k + j];

    // Tile x of this thread: rows 2A, 2A + 1 and columns 2B, 2B + 1 of the
    // Gram, B <= A, tile number A (A + 1) / 2 + B (an index past k is read
    // clamped and not written).  Every entry is summed by one thread over
    // the rows in order, as sum_r fma(P(r, a), P(r, b), s); its mirror has
    // the same bits.
    const int kh = (k + 1) / 2;
    const int ntile = kh * (kh + 1) / 2;
    // tile row A of tile ti, whose tile column is ti - A (A + 1) / 2
    // (recomputed where used: fewer live registers through the eigen-solves)
    auto tile_a = [](int ti) {
        int A = (int)((sqrt(8.0 * ti + 1.0) - 1.0) * 0.5);
        while ((A + 1) * (A + 2) / 2 <= ti) ++A;
        while (A * (A + 1) / 2 > ti) --A;
        return A;
    };
    constexpr int NT = TPT > 0 ? TPT : 1;
    double acc[NT][4];
    // Two passes over the kept rows.  Pass 0: G_P = P^T P.  Pass 1, after the
    // first eigen-solve: G_Y = Y^T Y with Y = P W1 recomputed from the rows,
    // so the singular values of P come out with relative accuracy.
    for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
        for (int x = 0; x < NT; ++x)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[x][v] = 0.0;
        for (int r0 = 0; r0 < m; r0 += RB) {
            const int nr = min(RB, m - r0);
            __syncthreads();
            for (int e = tid; e < nr * k; e += kThreads) {
                const int a = e % k;
                Us[e] = (double)Ub[(int64_t)r0 * k + e] * sblk[a];
            }
            __syncthreads();
            const double *R = Us;
            if (pass == 1) {
                if constexpr (TPT == 0) {
                    for (int e = tid; e < nr * k; e += kThreads) {
                        const int rr = e / k, j = e % k;
                        double s = 0.0;
                        for (int a = 0; a < k; ++a) s = fma(Us[rr * k + a], W1[a * ld + j], s);
                        Ys[e] = s;
                    }
                } else {
                    // Y = P W1 in 2 x 2 tiles (rows i0, i0 + 1; columns j0, j0 + 1),
                    // each output summed over a in order
                    const int ntc = (k + 1) / 2;
                    for (int t = tid; t < ((nr + 1) / 2) * ntc; t += kThreads) {
                        const int i0 = 2 * (t / ntc), j0 = 2 * (t % ntc);
                        const int i1 = min(i0 + 1, nr - 1), j1 = min(j0 + 1, k - 1);
                        double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
                        for (int a = 0; a < k; ++a) {
                            const double u0 = Us[i0 * k + a], u1 = Us[i1 * k + a];
                            const double w0 = W1[a * ld + j0], w1 = W1[a * ld + j1];
                            s00 = fma(u0, w0, s00);
                            s01 = fma(u0, w1, s01);
                            s10 = fma(u1, w0, s10);
                            s11 = fma(u1, w1, s11);
                        }
                        Ys[i0 * k + j0] = s00;
                        if (j0 + 1 < k) Ys[i0 * k + j0 + 1] = s01;
                        if (i0 + 1 < nr) {
                            Ys[(i0 + 1) * k + j0] = s10;
                            if (j0 + 1 < k) Ys[(i0 + 1) * k + j0 + 1] = s11;
                        }
                    }
                }
                __syncthreads();
                R = Ys;
            }
            if constexpr (TPT == 0) {
                if (tid < k * k) {
                    const int a = tid / k, b = tid % k;
                    double s = acc[0][0];
                    for (int rr = 0; rr < nr; ++rr) s = fma(R[rr * k + a], R[rr * k + b], s);
                    acc[0][0] = s;
                }
            } else {
#pragma unroll
                for (int x = 0; x < TPT; ++x) {
                    const int ti = tid + x * kThreads;
                    if (ti < ntile) {
                        const int A = tile_a(ti);
                        const int a0 = 2 * A, a1 = min(a0 + 1, k - 1);
                        const int b0 = 2 * (ti - A * (A + 1) / 2), b1 = min(b0 + 1, k - 1);
                        double s00 = acc[x][0], s01 = acc[x][1], s10 = acc[x][2], s11 = acc[x][3];
                        for (int rr = 0; rr < nr; ++rr) {
                            const double *row = R + rr * k;
                            const double p0 = row[a0], p1 = row[a1], q0 = row[b0], q1 = row[b1];
                            s00 = fma(p0, q0, s00);
                            s01 = fma(p0, q1, s01);
                            s10 = fma(p1, q0, s10);
                            s11 = fma(p1, q1, s11);
                        }
                        acc[x][0] = s00;
                        acc[x][1] = s01;
                        acc[x][2] = s10;
                        acc[x][3] = s11;
                    }
                }
            }
        }
        __syncthreads();
        // pass 0 starts W1 at the identity; pass 1 applies its rotations to
        // W1 itself, which leaves V~ = W1 J there
        if constexpr (TPT == 0) {
            if (tid < k * k) G[(tid / k) * ld + tid % k] = acc[0][0];
        } else {
#pragma unroll
            for (int x = 0; x < TPT; ++x) {
                const int ti = tid + x * kThreads;
                if (ti < ntile) {
                    const int A = tile_a(ti);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int a = 2 * A + v / 2, b = 2 * (ti - A * (A + 1) / 2) + v % 2;
                        if (a < k && b < k) {
                            G[a * ld + b] = acc[x][v];
                            G[b * ld + a] = acc[x][v];
                        }
                    }
                }
            }
        }
        if (pass == 0)
            for (int e = tid; e < k * k; e += kThreads) W1[(e / k) * ld + e % k] = (e / k == e % k) ? 1.0 : 0.0;
        __syncthreads();
        const int sweeps = sym_jacobi(G, W1, k, ld, cs_sh, sn_sh, dp_sh, dq_sh, &flag_sh, &tr_sh);
        if (sweeps < 0 && tid == 0) atomicOr(conv_flag, 1);
    }
    for (int j = tid; j < k; j += kThreads) sig[j] = sqrt(fmax(G[j * ld + j], 0.0));
    __syncthreads();                          // sig holds G's diagonal; V~ is in W1
    double smax = 0.0;
    for (int j = 0; j < k; ++j) smax = fmax(smax, sig[j]);
    // kept triplets: numerically non-zero and within the xi rank of Eq. (1)
    // over all k singular values of P (its whole spectrum), summed in
    // descending order
    for (int j = tid; j < k; j += kThreads) {
        int p = 0;
        for (int i = 0; i < k; ++i) p += (sig[i] > sig[j]) || (sig[i] == sig[j] && i < j);
        pinv[p] = j;
    }
    __syncthreads();
    double total = 0.0;
    for (int i = 0; i < k; ++i) total += sig[pinv[i]] * sig[pinv[i]];
    for (int j = tid; j < k; j += kThreads) {
        int prank = 0;
        for (int i = 0; i < k; ++i) prank += (sig[i] > sig[j]) || (sig[i] == sig[j] && i < j);
        bool kp = sig[j] > rank_tol * smax && sig[j] > 0.0;
        if (kp && xi > 0.0 && xi < 1.0 && total > 0.0) {
            double run = 0.0;
            for (int i = 0; i < prank; ++i) run += sig[pinv[i]] * sig[pinv[i]];
            kp = run < xi * total;
        }
        pkeep[j] = kp ? 1 : 0;
    }
    __syncthreads();

    // stack rows: Mp[j] = sigma~_j (V_(i) v~_j)^T = sigma~_j sum_l v~_lj V_(i)^T[l]
    const TU *Vt = static_cast<const TU *>(st.Vt) + pc.blk * k * st.c;
    double *Mrows = Mp + (int64_t)pc.t_idx * k * c;
    for (int e = tid; e < k * c; e += kThreads) {
        const int j = e / c, col = e % c;
        double s = 0.0;
        for (int l = 0; l < k; ++l) s = fma(W1[l * ld + j], (double)Vt[(int64_t)l * c + col], s);
        Mrows[e] = pkeep[j] ? sig[j] * s : 0.0;
    }
    // T = Sigma_(i) V~ Sigma~^+  (k x k, row-major)
    double *Tp = T + (int64_t)pc.t_idx * k * k;
    for (int e = tid; e < k * k; e += kThreads) {
        const int a = e / k, j = e % k;
        Tp[e] = pkeep[j] ? sblk[a] * W1[a * ld + j] / sig[j] : 0.0;
    }
}

}  // namespace

hipError_t set_sweep_cap(int cap)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(d_sweep_cap), &cap, sizeof(int), 0, hipMemcpyHostToDevice);
}

hipError_t launch_finalize(int c, int k, const Prob *probs, int nprob, int kk_max,
                           const double *GYpart, double *Vk, double *F, double rank_tol,
                           const double *const *gsrc, const double *const *msrc, double xi,
                           int *conv_flag, hipStream_t stream)
{
    if (nprob <= 0) return hipSuccess;
    if (kk_max < 1 || kk_max > kMaxK) return hipErrorInvalidValue;
    timing_begin("finalize", stream);
    const size_t lds = (size_t)(2 * kk_max * (kk_max + 1) + kFinRows * kk_max) * sizeof(double);
    static size_t cur = 0;
    {
        hipError_t e = ensure_lds((const void *)finalize_kernel, lds, cur);
        if (e != hipSuccess) return e;
    }
    finalize_kernel<<<nprob, kThreads, lds, stream>>>(c, k, probs, GYpart, Vk, F, rank_tol, kk_max,
                                                      gsrc, msrc, xi, conv_flag);
    hipError_t e = hipGetLastError();
    timing_end("finalize", stream);
    return e;
}

namespace {

template <int TPT>
hipError_t run_partial(StoreView st, const Piece *pieces, const int32_t *pidx, int npartial,
                       double *Mp, double *T, double rank_tol, double xi, int *conv_flag,
                       size_t lds, hipStream_t stream)
{
    static size_t cur_f = 0, cur_d = 0;   // one limit per instantiation
    hipError_t e = st.f32 ? ensure_lds((const void *)partial_kernel<float, TPT>, lds, cur_f)
                          : ensure_lds((const void *)partial_kernel<double, TPT>, lds, cur_d);
    if (e != hipSuccess) return e;
    if (st.f32)
        partial_kernel<float, TPT><<<npartial, kThreads, lds, stream>>>(st, pieces, pidx, Mp, T,
                                                                        rank_tol, xi, conv_flag);
    else
        partial_kernel<double, TPT><<<npartial, kThreads, lds, stream>>>(st, pieces, pidx, Mp, T,
                                                                         rank_tol, xi, conv_flag);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_partial(StoreView st, const Piece *pieces, const int32_t *pidx, int npartial,
                          double *Mp, double *T, double rank_tol, double xi, int *conv_flag,
                          hipStream_t stream)
{
    if (npartial <= 0) return hipSuccess;
    if (st.k < 1 || st.k > kMaxK) return hipErrorInvalidValue;
    timing_begin("partial", stream);
    const size_t lds = (size_t)(2 * st.k * (st.k + 1) + 2 * partial_rows(st.k) * st.k) * sizeof(double);
    const int kh = (st.k + 1) / 2;
    const int need = (kh * (kh + 1) / 2 + kThreads - 1) / kThreads;   // 2 x 2 tiles per thread
    hipError_t e;
    if (st.k < kPartialTileK) e = run_partial<0>(st, pieces, pidx, npartial, Mp, T, rank_tol, xi, conv_flag, lds, stream);
    else if (need <= 1) e = run_partial<1>(st, pieces, pidx, npartial, Mp, T, rank_tol, xi, conv_flag, lds, stream);
    else if (need <= 2) e = run_partial<2>(st, pieces, pidx, npartial, Mp, T, rank_tol, xi, conv_flag, lds, stream);
    else e = run_partial<3>(st, pieces, pidx, npartial, Mp, T, rank_tol, xi, conv_flag, lds, stream);
    timing_end("partial", stream);
    return e;
}

}  // namespace zs
