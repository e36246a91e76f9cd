// Leading eigenvectors of a symmetric positive semi-definite c x c Gram matrix
// by tridiagonalisation, one work-group per matrix (c <= 128).  With more
// matrices than CUs a work-group has 512 threads and keeps under half of a
// CU's LDS and registers, so two matrices share a CU and each one's barrier
// and latency stalls are filled by the other's work; with fewer, 1,024 threads
// give each matrix a whole CU.  Both forms round identically, so a problem's
// result does not depend on how many are solved together.
//
// First stage of every rank-k SVD of the method (the block SVDs of the
// storage phase and the SVD of each query's stacked matrix).  Only the span of
// the kk leading eigenvectors is used: the Rayleigh-Ritz stage that follows
// recomputes the singular values from the data with relative accuracy.
//
//   1. G <- the problem's Gram terms (fixed order), as in the Jacobi variant.
//   2. Householder tridiagonalisation Q^T G Q = T (Golub & Van Loan 8.3.1),
//      the reflector vectors packed one after another.
//   3. The kk largest eigenvalues of T by multisection on Sturm counts
//      (groups of up to 64 threads per eigenvalue).
//   4. Eigenvectors of T by inverse iteration (tridiagonal LU with partial
//      pivoting, two solves, one thread per cluster of eigenvalues closer
//      than 1e-9 ||T||, Gram-Schmidt inside a cluster: the approach of
//      LAPACK's stein).
//   5. Back-transformation x = Q z (the reflectors are parked in the
//      problem's own output slot, which is large enough for them while
//      c <= 2 kMaxK + 1), then two passes of classical Gram-Schmidt
//      over the kk vectors (a vector that collapses is replaced by the next
//      unit vector, which can only happen inside a degenerate eigenspace).
// The total work is O(c^3) with a small constant, against O(50 c^3) for
// one-sided Jacobi.
#include <atomic>
#include <cstdio>
#include <type_traits>

#include "zs_internal.h"
#include "wave.h"

namespace zs {
namespace {

// Partial sums of the reduction: the rows of wave w of a 1,024-thread
// work-group (w + 16 m) are the even-m rows of wave w mod 8 of a 512-thread
// one (w + 8 m), so that form keeps two FMA chains per wave and the sums agree
// bit for bit.
constexpr int kParts = 16;
// Dynamic LDS of one work-group, at most: two fit a CU's 160 KiB together
// with their static LDS.
constexpr int kLdsBudget = 10112;          // doubles

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
// then one region of `region` doubles.  The matrix itself never enters LDS:
// each thread keeps its elements in registers during the tridiagonal
// reduction, and the Householder vectors go to global memory.  The region is
// first the reduction's scratch (wave partials of A v, two v buffers, p, wave
// dot partials) and the staging of Partial-SVD rows, then the eigenvector block
// Z (c x kk) followed by the inverse-iteration arrays (two length-c arrays per
// solver lane).
template <int NMAX, int NTH>
struct TriLayout {
    static constexpr int kWaves = NTH / 64;
    static constexpr int FIXED = 4 * NMAX + kMaxK;
    static constexpr int SCR = kWaves * NMAX + 3 * NMAX + kParts;
    static_assert(SCR >= 8 * NMAX, "row staging of step 1 must fit the scratch");
    static_assert(NMAX <= 128, "two 64-bit words of pivot swaps per solver lane");
    static_assert((NMAX - 1) * NMAX / 2 <= NMAX * kMaxK, "reflectors fit the output slot");
    // region for c and a largest kk of k: all of Z, and as many solver lanes
    // (up to one per eigenvalue) as the budget leaves room for, at least one
    static int region(int c, int k)
    {
        const int room = kLdsBudget - FIXED - c * k;
        int nt = room / (2 * c);
        nt = nt < 1 ? 1 : (nt > k ? k : nt);
        const int need = c * k + 2 * c * nt;
        return need > SCR ? need : SCR;
    }
    static size_t bytes(int region) { return (size_t)(FIXED + region) * sizeof(double); }
};

template <int NMAX, int NTH>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4)))
void eig_tri_kernel(int c, int k, int region, const Prob *__restrict__ probs,
                    const double *const *__restrict__ gsrc, const double *const *__restrict__ msrc,
                    double *__restrict__ Vk)
{
    constexpr int kWaves = NTH / 64;
    constexpr int kSplit = kParts / kWaves;        // FMA chains per wave (1 or 2)
    static_assert(kSplit == 1 || kSplit == 2, "512 or 1,024 threads");
    constexpr int RPW = NMAX / kWaves;             // matrix rows per wave
    static_assert(RPW % kSplit == 0, "rows split evenly over the chains");
    constexpr int CPL = (NMAX + 63) / 64;          // matrix columns per lane
    constexpr int MR = 8;                          // rows of a Partial-SVD term staged at once
    extern __shared__ __align__(16) double smem[];
    double *d = smem;
    double *e = d + NMAX;
    double *e2 = e + NMAX;
    double *tau = e2 + NMAX;
    double *lam = tau + NMAX;                      // kMaxK
    double *scr = lam + kMaxK;                     // region: scratch (phases 1-3), later Z
    __shared__ double sh_a, sh_b, sh_tnorm, sh_pivmin;
    __shared__ int cl_start[kMaxK + 1];
    __shared__ int sh_ncl;

    const Prob P = probs[blockIdx.x];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    const int kk = P.kk;
    // c x kk, row-major; before that the packed Householder vectors, of
    // (c - 1) c / 2 <= c kMaxK doubles
    double *out = Vk + (int64_t)blockIdx.x * c * kMaxK;
    double *hv = out;
    // packed Householder vector j starts at hoff(j); its entry 0 is 1
    auto hoff = [c](int j) { return j * (c - 1) - j * (j - 1) / 2; };

    // Matrix element (R, C), R = wave + kWaves m, C = lane + 64 s, lives in a[m][s]
    // of this thread; elements outside c x c are zero.
    double a[RPW][CPL];

    // ---- 1. G ------------------------------------------------------------------
#pragma unroll
    for (int m = 0; m < RPW; ++m)
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int R = wave + kWaves * m, C = lane + 64 * s;
            double v = 0.0;
            if (R < c && C < c)
                for (int g = 0; g < P.ng; ++g) v += gsrc[P.g0 + g][R * c + C];
            a[m][s] = v;
        }
    for (int mm = 0; mm < P.nm; ++mm) {
        const double *Rm = msrc[P.m0 + mm];
        double *Rs = scr;                          // MR x c
        for (int r0 = 0; r0 < k; r0 += MR) {
            const int nr = min(MR, k - r0);
            __syncthreads();
            for (int q = tid; q < nr * c; q += NTH) Rs[q] = Rm[(int64_t)r0 * c + q];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < RPW; ++m) {
                const int R = wave + kWaves * m;
                if (R >= c) continue;
#pragma unroll
                for (int s = 0; s < CPL; ++s) {
                    const int C = lane + 64 * s;
                    if (C >= c) continue;
                    double v = a[m][s];
                    for (int r = 0; r < nr; ++r) v = fma(Rs[r * c + R], Rs[r * c + C], v);
                    a[m][s] = v;
                }
            }
        }
    }

    // ---- 2. tridiagonalisation Q^T G Q = T ---------------------------------------
    // Step j annihilates row / column j beyond j+1 with H_j = I - tau_j v_j v_j^T
    // (v_j(j+1) = 1) and applies H_j to the trailing block from both sides:
    //   p = tau A v,  w = p - (tau/2)(p.v) v,  A <- A - v w^T - w v^T.
    // Row j+1 is final after step j; the wave that holds it derives d, e and the
    // next reflector from its registers while the other waves go on, so each
    // step has three barriers.  Reflectors are kept in absolute indexing (zero
    // outside (j, c)) in two alternating buffers.
    double *part = scr;                            // kWaves x NMAX wave partials of A v
    double *vbuf = part + kWaves * NMAX;           // 2 x NMAX
    double *psh = vbuf + 2 * NMAX;                 // NMAX
    double *kpart = psh + NMAX;                    // kParts
    // Called by the wave that holds row jj once that row is final: x[s] is its
    // element (jj, lane + 64 s).  Sets d_jj and, below the last two rows, the
    // reflector of row jj (tau, e and the vector, also packed for later).
    auto row_final = [&](int jj, const double (&x)[CPL]) {
        double ss = 0.0;
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int C = lane + 64 * s;
            if (C > jj + 1 && C < c) ss = fma(x[s], x[s], ss);
        }
        ss = wave_sum64(ss);
        auto elem = [&](int C) {                   // x at column C (C uniform), from its lane
            double v = x[0];
#pragma unroll
            for (int s = 1; s < CPL; ++s)
                if ((C >> 6) == s) v = x[s];
            return readlane_d(v, C & 63);
        };
        const double alpha = jj + 1 < c ? elem(jj + 1) : 0.0;
        const double dj = elem(jj);
        if (lane == 0) d[jj] = dj;
        if (jj + 2 < c) {
            double t = 0.0, beta = alpha, scal = 0.0;
            if (ss > 0.0) {
                const double mu = sqrt(alpha * alpha + ss);
                beta = alpha <= 0.0 ? mu : -mu;
                t = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            double *vn = vbuf + ((jj & 1) * NMAX);
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                const int C = lane + 64 * s;
                if (C >= NMAX) continue;
                const double v = C == jj + 1 ? 1.0 : (C > jj + 1 && C < c ? x[s] * scal : 0.0);
                vn[C] = v;
                if (C > jj && C < c) hv[hoff(jj) + C - jj - 1] = v;
            }
            if (lane == 0) {
                tau[jj] = t;
                e[jj] = beta;
            }
        } else if (jj + 2 == c) {
            if (lane == 0) e[jj] = alpha;          // the last off-diagonal entry
        }
    };
    // the wave holding row jj copies it out of its registers (unrolled selects)
    auto take_row = [&](int jj, double (&x)[CPL]) {
#pragma unroll
        for (int s = 0; s < CPL; ++s) x[s] = 0.0;
#pragma unroll
        for (int m = 0; m < RPW; ++m)
            if (wave + kWaves * m == jj)
#pragma unroll
                for (int s = 0; s < CPL; ++s) x[s] = a[m][s];
    };

    if (wave == 0) {
        double x[CPL];
        take_row(0, x);
        row_final(0, x);
    }
    if (c == 2 && wave == 1) {
        double x[CPL];
        take_row(1, x);
        const double d1 = readlane_d(x[0], 1);
        if (lane == 0) d[1] = d1;
    }
    // Step j only touches the trailing block (j, c): v and w are zero outside
    // it, so the register rows m < M0 (rows below kWaves M0) and the 64-column
    // chunks s < S0 would only add exact zeros once j reaches them.  The
    // steps run in phases with compile-time M0, S0 (no branches in the
    // unrolled loops) that leave those registers out: the same bits with less
    // per-step element work.
    auto step = [&](int j, auto m0c, auto s0c) {
        constexpr int M0 = decltype(m0c)::value, S0 = decltype(s0c)::value;
        __syncthreads();                           // v_j and tau_j are visible
        const double *vc = vbuf + (j & 1) * NMAX;
        const double t = tau[j];
        // v is zero outside (j, c), so rows and columns outside the live block
        // contribute nothing and need no tests.
        // (the row entries of v and w are read from LDS where they are used,
        // which keeps the registers for the matrix)
        double vcl[CPL];
#pragma unroll
        for (int s = 0; s < CPL; ++s) vcl[s] = vc[min(lane + 64 * s, NMAX - 1)];   // 0 below S0
        // partial A v over this wave's rows (A symmetric: column sums = row sums)
        // and this wave's share of v^T A v, in kSplit chains (rows w + kWaves m
        // with m of one parity each)
        double pp[kSplit][CPL];
#pragma unroll
        for (int x = 0; x < kSplit; ++x)
#pragma unroll
            for (int s = 0; s < CPL; ++s) pp[x][s] = 0.0;
#pragma unroll
        for (int m = M0; m < RPW; ++m) {
            const double vr = vc[wave + kWaves * m];
#pragma unroll
            for (int s = S0; s < CPL; ++s) pp[m % kSplit][s] = fma(a[m][s], vr, pp[m % kSplit][s]);
        }
#pragma unroll
        for (int x = 0; x < kSplit; ++x) {
            double vav = 0.0;
#pragma unroll
            for (int s = S0; s < CPL; ++s)
                if (lane + 64 * s < c) vav = fma(pp[x][s], vcl[s], vav);
            vav = wave_sum64(vav);
            if (lane == 0) kpart[wave + kWaves * x] = vav;
        }
        // the first level of the pairwise tree over kParts partials (parts w and
        // w + 8) is the sum of this wave's two chains
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const double ps = kSplit == 2 ? pp[0][s] + pp[kSplit - 1][s] : pp[0][s];
            if (lane + 64 * s < NMAX) part[wave * NMAX + lane + 64 * s] = ps;
        }
        __syncthreads();
        // p = tau A v (pairwise sum of the wave partials)
        if (tid < c) {
            double h[kWaves];
#pragma unroll
            for (int w = 0; w < kWaves; ++w) h[w] = part[w * NMAX + tid];
#pragma unroll
            for (int st = kWaves / 2; st >= 1; st /= 2)
#pragma unroll
                for (int w = 0; w < st; ++w) h[w] += h[w + st];
            psh[tid] = t * h[0];
        }
        double kv[kParts];
#pragma unroll
        for (int w = 0; w < kParts; ++w) kv[w] = kpart[w];
#pragma unroll
        for (int st = kParts / 2; st >= 1; st /= 2)
#pragma unroll
            for (int w = 0; w < st; ++w) kv[w] += kv[w + st];
        const double K = 0.5 * t * t * kv[0];      // (tau/2) p.v with p.v = tau v^T A v
        __syncthreads();
        // A <- A - v w^T - w v^T, w = p - K v (zero outside the live block)
        double wcol[CPL];
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int C = lane + 64 * s;
            const double pc = psh[min(C, NMAX - 1)];
            wcol[s] = (C > j && C < c) ? pc - K * vcl[s] : 0.0;
        }
#pragma unroll
        for (int m = M0; m < RPW; ++m) {
            const int R = wave + kWaves * m;
            const double vr = vc[R], pr = psh[R];   // unconditional reads: a select, no branch
            const double wr = (R > j && R < c) ? pr - K * vr : 0.0;
#pragma unroll
            for (int s = S0; s < CPL; ++s) {
                a[m][s] = fma(-vr, wcol[s], a[m][s]);
                a[m][s] = fma(-wr, vcl[s], a[m][s]);
            }
        }
        // row j+1 is final: its holder prepares step j+1
        if (wave == (j + 1) % kWaves) {
            double x[CPL];
            take_row(j + 1, x);
            row_final(j + 1, x);
        }
        if (j + 3 == c && wave == (c - 1) % kWaves) {   // last step: row c-1 is final too
            double x[CPL];
            take_row(c - 1, x);
            double v = x[0];
#pragma unroll
            for (int s = 1; s < CPL; ++s)
                if (((c - 1) >> 6) == s) v = x[s];
            const double xd = readlane_d(v, (c - 1) & 63);
            if (lane == 0) d[c - 1] = xd;
        }
    
    };
    {
        // two phases: all registers while j < NMAX / 2, then only the trailing
        // quarter (rows and columns >= NMAX / 2); more phases make the
        // 512-thread form spill
        using std::integral_constant;
        const int jend = c - 2;
        int j = 0;
        for (; j < jend && j < NMAX / 2; ++j) step(j, integral_constant<int, 0>(), integral_constant<int, 0>());
        for (; j < jend; ++j)
            step(j, integral_constant<int, NMAX / 2 / kWaves>(), integral_constant<int, (NMAX / 2) / 64>());
    }
    __syncthreads();
    if (tid == 0) {
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
    for (int i = tid; i + 1 < c; i += NTH) e2[i] = e[i] * e[i];
    __syncthreads();
    const double tnorm = sh_tnorm, pivmin = sh_pivmin;

    if (tnorm == 0.0) {                   // zero matrix: any orthonormal basis
        for (int q = tid; q < c * kk; q += NTH) out[q] = (q / kk == q % kk) ? 1.0 : 0.0;
        return;
    }

    // ---- 3. the kk largest eigenvalues: multisection on Sturm counts ---------------
    // Groups of G lanes inside one wave share an eigenvalue: each lane counts
    // the eigenvalues below its point, a ballot finds the first point whose
    // count exceeds the wanted index, and the interval shrinks G+1 times per
    // round.  Waves run their rounds independently.  A Sturm count is a chain
    // of c divisions, so G is chosen to keep about 256 lanes busy (one wave per
    // SIMD): more lanes would make the rounds issue-bound, fewer would add
    // rounds of the same latency.
    {
        const int G = kk <= 4 ? 64 : (kk <= 8 ? 32 : (kk <= 16 ? 16 : (kk <= 32 ? 8 : 4)));
        const int gpw = 64 / G;                    // groups per wave
        const int gb = (lane / G) * G;             // first lane of this lane's group
        const int grp = wave * gpw + lane / G;     // eigenvalue, largest first
        const int mem = lane - gb;
        const int m = c - 1 - grp;                 // its ascending index
        const double atol = 4.0 * __DBL_EPSILON__ * tnorm + 2.0 * pivmin;
        double lo = sh_a, hi = sh_b;
        bool live = grp < kk;
        for (int it = 0; it < 80; ++it) {
            if (!__any(live)) break;               // wave-uniform exit
            const double x = lo + (hi - lo) * (double)(mem + 1) / (double)(G + 1);
            double q = d[0] - x;
            if (fabs(q) < pivmin) q = -pivmin;
            int cnt = q < 0.0;
            // the next row's d and e^2 are loaded one step ahead, so that the LDS
            // latency stays off the recurrence
            double dn = d[min(1, c - 1)], en = e2[0];
            for (int i = 1; i < c; ++i) {
                const double di = dn, ei = en;
                dn = d[min(i + 1, c - 1)];
                en = e2[min(i, c - 2)];
                q = (di - x) - ei / q;
                if (fabs(q) < pivmin) q = -pivmin;
                cnt += q < 0.0;
            }
            const uint64_t above = __ballot(cnt > m);
            const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
            const uint64_t bits = (above >> gb) & gmask;
            const int f = bits ? __builtin_ctzll(bits) : G;   // first point above
            const double xf = __shfl(x, gb + min(f, G - 1), 64);
            const double xp = __shfl(x, gb + max(f - 1, 0), 64);
            if (live) {
                if (f < G) hi = xf;
                if (f > 0) lo = xp;
                if (hi - lo <= atol) live = false;
            }
        }
        if (grp < kk && mem == 0) lam[grp] = 0.5 * (lo + hi);
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

    // ---- 4. inverse iteration: one lane of wave 0 per cluster, members in order ----
    //      Z (c x kk) starts the region.  Each solver lane keeps the U factor of
    //      T - lambda I in two length-c arrays after Z, interleaved by lane
    //      (element i at i * NT + lane): the reciprocal diagonal and the first
    //      superdiagonal.  The second superdiagonal is e(i+1) where row i was
    //      swapped and zero elsewhere, so a bit per row in registers stands for
    //      it.  The eliminated right-hand side overwrites z in place.  The
    //      recurrences load the next row of T and of z one step ahead, so that
    //      LDS latency stays off the dependence chain.
    double *Z = scr;
    if (wave == 0) {
        double *lu = Z + c * kk;
        const int NT = min((region - c * kk) / (2 * c), 64);
        const int ncl = sh_ncl;
        const double pivfloor = __DBL_EPSILON__ * tnorm;
        for (int cb = 0; cb < ncl; cb += NT) {
            const int cl = cb + lane;
            const bool act = lane < NT && cl < ncl;
            double *u1 = lu + min(lane, NT - 1), *u2 = u1 + c * NT;
            const int g0 = act ? cl_start[cl] : 0, g1 = act ? cl_start[cl + 1] : 0;
            // members of every lane's cluster in step (lanes with fewer idle)
            int gmax = g1 - g0;
            for (int off = 32; off >= 1; off >>= 1) gmax = max(gmax, __shfl_xor(gmax, off, 64));
            for (int gi = 0; gi < gmax; ++gi) {
                const bool on = gi < g1 - g0;
                const int g = on ? g0 + gi : 0;
                const double lmb = on ? lam[g] : 0.0;
                double *z = Z + g;                 // column g, stride kk
                int attempt = 0;
                if (on)
                    for (int i = 0; i < c; ++i) z[i * kk] = start_value(i, g, attempt);
                for (int it = 0; it < 2; ++it) {
                    if (on) {
                        // LU with partial pivoting of T - lmb I, applied to z.  The
                        // next row of T and of z is loaded one step ahead.
                        double p0 = d[0] - lmb, p1 = c > 1 ? e[0] : 0.0, r = z[0];
                        double svn = e[0], ddn = d[min(1, c - 1)], een = e[min(1, c - 1)];
                        double znn = z[min(1, c - 1) * kk];
                        uint64_t swl = 0, swh = 0;   // rows 0-63 and 64-127 swapped
                        for (int i = 0; i + 1 < c; ++i) {
                            const double sv = svn, dd = ddn - lmb, ee = (i + 2 < c) ? een : 0.0;
                            const double zn = znn;
                            const int i2 = min(i + 2, c - 1);
                            svn = e[i + 1];
                            ddn = d[i2];
                            een = e[i2];
                            znn = z[i2 * kk];
                            // pivot on the larger of p0 and the subdiagonal entry
                            const bool swap = fabs(sv) > fabs(p0);
                            double piv = p0;
                            if (fabs(piv) < pivfloor) piv = piv < 0.0 ? -pivfloor : pivfloor;
                            const double den = swap ? sv : piv;
                            const double inv = 1.0 / den;
                            const double mlt = (swap ? p0 : sv) * inv;
                            u1[i * NT] = inv;
                            u2[i * NT] = swap ? dd : p1;
                            const uint64_t bit = (uint64_t)swap << (i & 63);
                            if (i < 64) swl |= bit;
                            else swh |= bit;
                            z[i * kk] = swap ? zn : r;
                            const double np0 = swap ? p1 - mlt * dd : dd - mlt * p1;
                            const double np1 = swap ? -mlt * ee : ee;
                            r = swap ? r - mlt * zn : zn - mlt * r;
                            p0 = np0;
                            p1 = np1;
                        }
                        if (fabs(p0) < pivfloor) p0 = p0 < 0.0 ? -pivfloor : pivfloor;
                        double y2 = 0.0, y1 = r / p0;
                        z[(c - 1) * kk] = y1;
#pragma unroll 4
                        for (int i = c - 2; i >= 0; --i) {
                            const bool sw = (((i < 64 ? swl : swh) >> (i & 63)) & 1) != 0;
                            const double u3 = (sw && i + 2 < c) ? e[i + 1] : 0.0;
                            const double y = (z[i * kk] - u2[i * NT] * y1 - u3 * y2) * u1[i * NT];
                            z[i * kk] = y;
                            y2 = y1;
                            y1 = y;
                        }
                        // Gram-Schmidt against earlier members of the cluster, normalise
                        for (int h = g0; h < g; ++h) {
                            const double *zh = Z + h;
                            double sd = 0.0;
                            for (int i = 0; i < c; ++i) sd = fma(zh[i * kk], z[i * kk], sd);
                            for (int i = 0; i < c; ++i) z[i * kk] -= sd * zh[i * kk];
                        }
                        double n0 = 0.0, n1 = 0.0;
#pragma unroll 4
                        for (int i = 0; i + 1 < c; i += 2) {
                            n0 = fma(z[i * kk], z[i * kk], n0);
                            n1 = fma(z[(i + 1) * kk], z[(i + 1) * kk], n1);
                        }
                        if (c & 1) n0 = fma(z[(c - 1) * kk], z[(c - 1) * kk], n0);
                        const double nrm = n0 + n1;
                        if (!(nrm > 0.0) || !isfinite(nrm)) {
                            ++attempt;               // restart from another vector
                            for (int i = 0; i < c; ++i) z[i * kk] = start_value(i, g, attempt);
                            continue;
                        }
                        const double sc = 1.0 / sqrt(nrm);
                        for (int i = 0; i < c; ++i) z[i * kk] *= sc;
                    }
                }
            }
        }
    }
    __syncthreads();

    // ---- 5. back-transformation x = H_0 H_1 ... H_{c-3} z, columns in registers ----
    //      The reflectors are read from global memory (just written, so from
    //      cache) kPre steps ahead of their use.
    {
        constexpr int CPW = kMaxK / kWaves;        // columns per wave, at most
        constexpr int kPre = 4;
        double z0[CPW], z1[CPW];
        const int ncol = (kk - wave + kWaves - 1) / kWaves;
#pragma unroll
        for (int u = 0; u < CPW; ++u) {
            const int g = wave + u * kWaves;
            z0[u] = (u < ncol && lane < c) ? Z[lane * kk + g] : 0.0;
            z1[u] = (u < ncol && lane + 64 < c) ? Z[(lane + 64) * kk + g] : 0.0;
        }
        // entries (lane, lane + 64) of reflector j, zero outside (j, c)
        auto vload = [&](int j, double &v0, double &v1) {
            const int i0 = lane - (j + 1), i1 = lane + 64 - (j + 1);
            const double *vj = hv + hoff(max(j, 0));
            v0 = (j >= 0 && i0 >= 0 && lane < c) ? vj[i0] : 0.0;
            v1 = (j >= 0 && i1 >= 0 && lane + 64 < c) ? vj[i1] : 0.0;
        };
        if (ncol > 0) {
            double q0[kPre], q1[kPre];             // reflectors j, j-1, ..., j-kPre+1
#pragma unroll
            for (int p = 0; p < kPre; ++p) vload(c - 3 - p, q0[p], q1[p]);
            for (int j = c - 3; j >= 0; --j) {
                const double t = tau[j];
                const double v0 = q0[0], v1 = q1[0];
#pragma unroll
                for (int p = 0; p + 1 < kPre; ++p) {
                    q0[p] = q0[p + 1];
                    q1[p] = q1[p + 1];
                }
                vload(j - kPre, q0[kPre - 1], q1[kPre - 1]);
                if (t == 0.0) continue;
                double sv[CPW];
#pragma unroll
                for (int u = 0; u < CPW; ++u) sv[u] = fma(v0, z0[u], v1 * z1[u]);
#pragma unroll
                for (int u = 0; u < CPW; ++u)
                    if (u < ncol) sv[u] = wave_sum64(sv[u]);
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
                    sd = wave_sum64(sd);
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
                const double nrm2 = wave_sum64(sn);  // every wave computes the same norm
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

template <int NMAX, int NTH>
hipError_t run_eig_tri(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                       const double *const *msrc, double *Vk, hipStream_t stream)
{
    // every problem's kk is at most k
    const int region = TriLayout<NMAX, NTH>::region(c, k);
    const size_t lds = TriLayout<NMAX, NTH>::bytes(region);
    static size_t cur = 0;
    hipError_t e = ensure_lds((const void *)eig_tri_kernel<NMAX, NTH>, lds, cur);
    if (e != hipSuccess) return e;
    eig_tri_kernel<NMAX, NTH><<<nprob, NTH, lds, stream>>>(c, k, region, probs, gsrc, msrc, Vk);
    return hipGetLastError();
}

// Compute units of the current device (0 if the query fails), cached per device.
int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 0;
    }
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

// 512 threads and two matrices per CU, or 1,024 threads and one: both forms
// round identically, so the autotuner picks per shape; without a choice, two
// per CU once there are more matrices than CUs, else one.
template <int NMAX>
hipError_t run_eig_tri(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                       const double *const *msrc, double *Vk, hipStream_t stream)
{
    char key[64];
    snprintf(key, sizeof key, "c=%d k=%d n=%d", c, k, tune_bucket(nprob));
    const int dflt = nprob <= device_cus() ? 1 : 0;
    return tuned_launch("eig_tri_threads", key, 2, dflt, stream, [&](int v) {
        return v == 1 ? run_eig_tri<NMAX, 1024>(c, k, probs, nprob, gsrc, msrc, Vk, stream)
                      : run_eig_tri<NMAX, 512>(c, k, probs, nprob, gsrc, msrc, Vk, stream);
    });
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
