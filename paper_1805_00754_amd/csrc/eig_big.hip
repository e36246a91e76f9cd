// Leading eigenvectors of a symmetric positive semi-definite c x c Gram matrix
// for 128 < c <= 1024, one work-group of 1024 threads per matrix, with the
// matrix in a global scratch slot (L2 / Infinity Cache resident) and the
// vectors of each step in LDS.  Same method as the solver for c <= 128
// (eig_tri.hip), whose matrix fits in registers:
//
//   1. W <- the problem's Gram terms (tree nodes / block chunk Grams, then the
//      Grams of its Partial-SVD rows), in a fixed order.
//   2. Householder tridiagonalisation Q^T W Q = T, one reflector per step:
//      the reflector of row j (rows are contiguous, the matrix is kept
//      symmetric) is formed in LDS and saved over the dead part of row j;
//      p = t W22 v, W22 -= v w^T + w v^T.  The update of step j and the
//      product of step j+1 share one pass over the trailing rows: row j+1
//      (kept in LDS by the previous pass) is updated first and gives the next
//      reflector, then every other trailing row is updated and multiplied by
//      it while in registers (each wave takes several rows at a time, so
//      their loads overlap).
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

constexpr int NTH = 1024;
constexpr int kWaves = NTH / 64;
constexpr int kBigMax = 1024;             // largest c
constexpr int kWU = 8;                    // matrix entries per thread in flight in phase 1

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the work-group; red holds kWaves doubles.  All threads call it.
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

// VPL: vector entries per lane in phase 5 (c <= 64 VPL).
template <int VPL>
__global__ __launch_bounds__(NTH) void eig_big_kernel(int c, int k, const Prob *__restrict__ probs,
                                                      const double *const *__restrict__ gsrc,
                                                      const double *const *__restrict__ msrc,
                                                      double *__restrict__ scratch,
                                                      double *__restrict__ Vk)
{
    __shared__ double d[kBigMax], e[kBigMax], e2[kBigMax], tau[kBigMax];
    __shared__ double vbuf[2][kBigMax], wbuf[2][kBigMax];   // v and p / w of two steps
    __shared__ double rowb[kBigMax];      // the next row to reduce, from its diagonal on
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

    // ---- 1. W ------------------------------------------------------------------
    //      Each thread sums kWU entries at a time (independent loads in flight),
    //      each entry in the fixed term order.
    const int64_t cc = (int64_t)c * c;
    for (int64_t q0 = tid; q0 < cc; q0 += (int64_t)NTH * kWU) {
        double s[kWU];
#pragma unroll
        for (int x = 0; x < kWU; ++x) s[x] = 0.0;
        for (int g = 0; g < P.ng; ++g) {
            const double *src = gsrc[P.g0 + g];
#pragma unroll
            for (int x = 0; x < kWU; ++x) {
                const int64_t q = q0 + (int64_t)x * NTH;
                if (q < cc) s[x] += src[q];
            }
        }
#pragma unroll
        for (int x = 0; x < kWU; ++x) {
            const int64_t q = q0 + (int64_t)x * NTH;
            if (q < cc) W[q] = s[x];
        }
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

    // ---- 2. tridiagonalisation ---------------------------------------------------
    // Reflector of row jr (final, entries jr .. c-1 in rowb): tau, e, d of jr
    // and v (length c - jr - 1, v(0) = 1) into vdst and over the dead part of
    // row jr in W.
    auto make_reflector = [&](int jr, double *vdst) {
        const int n = c - jr - 1;
        double *rowj = W + (int64_t)jr * c;
        double part = 0.0;
        for (int i = tid + 1; i < n; i += NTH) part = fma(rowb[1 + i], rowb[1 + i], part);
        const double s = block_sum(part, red);
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
    // Step j runs with v_j = vbuf[j & 1] and p_j = t_j W22 v_j in wbuf[j & 1];
    // j = -1 only forms reflector 0 and p_0.  Row j+1 lives in rowb from the
    // pass of step j-1 on (the pass that updates it also keeps it there), so
    // its last update and its reflector take no global round trip.
    constexpr int RU = 4;                          // rows per wave in flight
    constexpr int CU = 4;                          // 64-column chunks per row in flight
    for (int i = tid; i < c; i += NTH) rowb[i] = W[i];   // row 0
    __syncthreads();
    for (int j = -1; j + 2 < c; ++j) {
        const int n1 = c - j - 1;                  // trailing size of step j
        const double *vc = vbuf[j & 1];
        double *wc = wbuf[j & 1];
        double *vn = vbuf[(j + 1) & 1];
        double *wn = wbuf[(j + 1) & 1];
        const double t = j >= 0 ? tau[j] : 0.0;
        const bool upd = t != 0.0;
        if (upd) {
            // w = p - K v, K = (t/2) p.v
            double pk = 0.0;
            for (int i = tid; i < n1; i += NTH) pk = fma(wc[i], vc[i], pk);
            const double K = 0.5 * t * block_sum(pk, red);
            for (int i = tid; i < n1; i += NTH) wc[i] -= K * vc[i];
            __syncthreads();
            // row j+1 first: it gives the next reflector
            const double v0 = vc[0], w0 = wc[0];
            for (int i = tid; i < n1; i += NTH) rowb[i] -= v0 * wc[i] + w0 * vc[i];
            __syncthreads();
        }
        const bool next = j + 3 < c;
        if (!next && tid == 0) {                   // row c-2 is final: d and e of it
            d[c - 2] = rowb[0];
            e[c - 2] = rowb[1];
        }
        if (next) {
            make_reflector(j + 1, vn);
            __syncthreads();
        }
        const double tn = next ? tau[j + 1] : 0.0;
        const bool dot = tn != 0.0;
        // rows j+2 .. c-1, columns j+2 .. c-1: update of step j, then p_{j+1}
        const int nr = n1 - 1;
        double *Wt = W + (int64_t)(j + 2) * c + j + 2;
        if (upd || dot) {
            for (int q0 = wave * RU; q0 < nr; q0 += kWaves * RU) {
                double vr[RU], wr[RU], acc[RU];
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const bool live = q0 + u < nr;
                    vr[u] = (upd && live) ? vc[q0 + u + 1] : 0.0;
                    wr[u] = (upd && live) ? wc[q0 + u + 1] : 0.0;
                    acc[u] = 0.0;
                }
                for (int i0 = 0; i0 < nr; i0 += 64 * CU) {
                    double vi[CU], wi[CU], vx[CU], x[RU][CU];
#pragma unroll
                    for (int h = 0; h < CU; ++h) {
                        const int ip = i0 + 64 * h + lane;
                        const bool in = ip < nr;
                        vi[h] = (upd && in) ? vc[ip + 1] : 0.0;
                        wi[h] = (upd && in) ? wc[ip + 1] : 0.0;
                        vx[h] = (dot && in) ? vn[ip] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < RU; ++u)
#pragma unroll
                        for (int h = 0; h < CU; ++h) {
                            const int ip = i0 + 64 * h + lane;
                            x[u][h] = (ip < nr && q0 + u < nr) ? Wt[(int64_t)(q0 + u) * c + ip] : 0.0;
                        }
#pragma unroll
                    for (int u = 0; u < RU; ++u)
#pragma unroll
                        for (int h = 0; h < CU; ++h) {
                            const int ip = i0 + 64 * h + lane;
                            if (upd) {
                                x[u][h] -= vr[u] * wi[h] + wr[u] * vi[h];
                                if (ip < nr && q0 + u < nr) Wt[(int64_t)(q0 + u) * c + ip] = x[u][h];
                            }
                            acc[u] = fma(x[u][h], vx[h], acc[u]);
                        }
                    if (q0 == 0)                   // row j+2, the next row to reduce
#pragma unroll
                        for (int h = 0; h < CU; ++h) {
                            const int ip = i0 + 64 * h + lane;
                            if (ip < nr) rowb[ip] = x[0][h];
                        }
                }
                if (dot) {
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        const double sdot = wave_sum64(acc[u]);
                        if (lane == 0 && q0 + u < nr) wn[q0 + u] = tn * sdot;
                    }
                }
            }
        } else {
            for (int i = tid; i < nr; i += NTH) rowb[i] = Wt[i];   // row j+2 as it is
        }
        __syncthreads();
    }
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
        constexpr int CPP = VPL <= 4 ? 4 : (VPL <= 8 ? 2 : 1);
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

    // ---- 6. classical Gram-Schmidt, twice -----------------------------------------
    for (int g = 0; g < kk; ++g) {
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
            const double nrm2 = block_sum(sn, red);
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
    if (c <= 256) eig_big_kernel<4><<<nprob, NTH, 0, stream>>>(c, k, probs, gsrc, msrc, scratch, Vk);
    else if (c <= 512) eig_big_kernel<8><<<nprob, NTH, 0, stream>>>(c, k, probs, gsrc, msrc, scratch, Vk);
    else eig_big_kernel<16><<<nprob, NTH, 0, stream>>>(c, k, probs, gsrc, msrc, scratch, Vk);
    hipError_t e = hipGetLastError();
    timing_end("eig", stream);
    return e;
}

}  // namespace zs
