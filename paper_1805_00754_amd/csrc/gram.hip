// Tall-skinny Gram panels: G = X^T X over a run of rows of X, accumulated in
// FP64 whatever the element type of X (double, float or bf16).
//
// Used for the block Gram G_i = A_(i)^T A_(i) of the storage phase and for the
// Gram of each query's stacked matrix M = [Sigma'_S V'_S^T; ...; Sigma'_E V'_E^T]
// (the stacked SVD of Alg. 2).  Each work-group owns one chunk of rows and one
// (16*TM) x (16*TM) output tile; rows are staged through LDS in panels of RB
// rows with coalesced loads, every thread accumulates a TM x TM register tile.
// Partial Grams of the chunks of one problem go to separate slots and are
// summed in a fixed order by the consumer, so results do not depend on how
// many other problems share the launch.
#include "zs_internal.h"

#include <cstdio>

namespace zs {
namespace {

template <int TM, typename TA>
__global__ __launch_bounds__(kThreads) void gram_kernel(const TA *__restrict__ X, int64_t ld,
                                                        int c, const Chunk *__restrict__ chunks,
                                                        double *__restrict__ Gpart)
{
    constexpr int TILE = 16 * TM;
    constexpr int RB = 16;
    __shared__ __align__(16) double Xi[RB][TILE];
    __shared__ __align__(16) double Xj[RB][TILE];

    const Chunk ch = chunks[blockIdx.x];
    const int ntile = (c + TILE - 1) / TILE;
    int idx = blockIdx.y, ti = 0;
    while (idx >= ntile - ti) { idx -= ntile - ti; ++ti; }
    const int tj = ti + idx;
    const int ci0 = ti * TILE, cj0 = tj * TILE;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;

    double acc[TM][TM];
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int n = 0; n < TM; ++n) acc[m][n] = 0.0;

    const TA *Xc = X + ch.x_off;
    for (int r0 = 0; r0 < ch.rows; r0 += RB) {
        for (int e = threadIdx.x; e < RB * TILE; e += kThreads) {
            const int rr = e / TILE, cc = e % TILE;
            const int row = r0 + rr;
            double vi = 0.0, vj = 0.0;
            if (row < ch.rows) {
                const TA *xr = Xc + (int64_t)row * ld;
                if (ci0 + cc < c) vi = load_as_double(xr, ci0 + cc);
                if (cj0 + cc < c) vj = load_as_double(xr, cj0 + cc);
            }
            Xi[rr][cc] = vi;
            Xj[rr][cc] = vj;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < RB; ++rr) {
            double a[TM], bb[TM];
#pragma unroll
            for (int m = 0; m < TM; ++m) {
                a[m] = Xi[rr][ty * TM + m];
                bb[m] = Xj[rr][tx * TM + m];
            }
#pragma unroll
            for (int m = 0; m < TM; ++m)
#pragma unroll
                for (int n = 0; n < TM; ++n) acc[m][n] = fma(a[m], bb[n], acc[m][n]);
        }
        __syncthreads();
    }

    double *G = Gpart + (int64_t)ch.slot * c * c;
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const int i = ci0 + ty * TM + m;
        if (i >= c) continue;
#pragma unroll
        for (int n = 0; n < TM; ++n) {
            const int j = cj0 + tx * TM + n;
            if (j >= c) continue;
            G[(int64_t)i * c + j] = acc[m][n];
            if (ti != tj) G[(int64_t)j * c + i] = acc[m][n];
        }
    }
}

}  // namespace

// Matrix-core form for c <= 128 (at most 8 blocks of 16 columns): one chunk
// per work-group column, G = sum over 4-row steps of F_i^T F_j, where F_b is
// the step's 4 x 16 slice of column block b.  With FP64 MFMA 16x16x4 the A
// operand A(i, s) = X(s, 16 ci + i) and the B operand B(s, j) = X(s, 16 cj + j)
// have the same lane layout (element (s, e) of a slice in lane e + 16 s), so
// one load per column block and step feeds every block product of the step.
// Only blocks ci <= cj are formed (the result is symmetric); wave w owns the
// block columns w and NB - 1 - w, which balances the work: NB + 1 blocks per
// wave for even NB.  D(i, j) sits in register i / 4 of lane j + 16 (i mod 4).
typedef double v4d __attribute__((ext_vector_type(4)));

template <int NBM, typename TA>
__global__ __launch_bounds__(kThreads) void gram_mfma_kernel(const TA *__restrict__ X, int64_t ld,
                                                             int c, const Chunk *__restrict__ chunks,
                                                             double *__restrict__ Gpart)
{
    const Chunk ch = chunks[blockIdx.x];
    const int nb = (c + 15) / 16;
    const int lane = threadIdx.x % 64;
    const int w = (int)blockIdx.y * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    if (2 * w > nb - 1) return;                    // no block column for this wave
    const int ca = w, cb = nb - 1 - w;             // owned block columns (ca <= cb)
    const bool two = cb != ca;
    const TA *Xc = X + ch.x_off;
    const int e = lane % 16, s4 = lane / 16;
    v4d acc_a[NBM], acc_b[NBM];
#pragma unroll
    for (int b = 0; b < NBM; ++b) {
        acc_a[b] = (v4d){0.0, 0.0, 0.0, 0.0};
        acc_b[b] = (v4d){0.0, 0.0, 0.0, 0.0};
    }
    // Steps of 4 rows, ST per half-iteration, in two register sets used in
    // turn: one set's loads are in flight while the other feeds the matrix
    // cores.  Every load is issued (row and column clamped, so no load sits
    // under a branch and no wait drains the other set); rows past the chunk
    // are zeroed by an exact multiply when they are used.
    constexpr int ST = NBM <= 8 ? 2 : 1;
    auto load = [&](int r0, double (&f)[ST][NBM]) {
#pragma unroll
        for (int q = 0; q < ST; ++q) {
            const int64_t r = min(r0 + 4 * q + s4, ch.rows - 1);
#pragma unroll
            for (int b = 0; b < NBM; ++b) f[q][b] = load_as_double(Xc, r * ld + min(16 * b + e, c - 1));
        }
    };
    auto steps = [&](int r0, double (&f)[ST][NBM]) {
#pragma unroll
        for (int q = 0; q < ST; ++q) {
            const double keep = r0 + 4 * q + s4 < ch.rows ? 1.0 : 0.0;
#pragma unroll
            for (int b = 0; b < NBM; ++b) f[q][b] *= keep;
            double fa = f[q][0], fb = f[q][0];
#pragma unroll
            for (int b = 1; b < NBM; ++b) {
                if (b == ca) fa = f[q][b];
                if (b == cb) fb = f[q][b];
            }
#pragma unroll
            for (int b = 0; b < NBM; ++b) {
                if (b <= ca) acc_a[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[q][b], fa, acc_a[b], 0, 0, 0);
                if (two && b <= cb)
                    acc_b[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[q][b], fb, acc_b[b], 0, 0, 0);
            }
        }
    };
    constexpr int H = 4 * ST;                      // rows per half-iteration
    double f1[ST][NBM], f2[ST][NBM];
    load(0, f1);
    for (int r0 = 0; r0 < ch.rows; r0 += 2 * H) {
        load(r0 + H, f2);                          // past the chunk: clamped, unused
        __builtin_amdgcn_sched_barrier(0);
        steps(r0, f1);
        if (r0 + H >= ch.rows) break;
        load(r0 + 2 * H, f1);
        __builtin_amdgcn_sched_barrier(0);
        steps(r0 + H, f2);
    }
    double *G = Gpart + (int64_t)ch.slot * c * c;
    auto put = [&](int bi, int bj, const v4d &d) {  // block (bi, bj) and its transpose
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * bi + 4 * v + lane / 16, j = 16 * bj + lane % 16;
            if (i < c && j < c) {
                G[(int64_t)i * c + j] = d[v];
                if (bi != bj) G[(int64_t)j * c + i] = d[v];
            }
        }
    };
#pragma unroll
    for (int b = 0; b < NBM; ++b) {
        if (b <= ca) put(b, ca, acc_a[b]);
        if (two && b <= cb) put(b, cb, acc_b[b]);
    }
}

// ------------------------------------------------------ FP32 / BF16 arithmetic
// The block Gram of the FP32 and BF16 modes on the matrix cores, widened to
// FP64 for the eigen-solver (which, like the refinement after it, stays in
// FP64):
//   BF16: v_mfma_f32_16x16x32_bf16.  bf16 input enters exactly; wider input
//         is rounded to bf16 (to nearest even; FP64 through FP32).
//   FP32: v_mfma_f32_16x16x4f32 on the input rounded to FP32.
// The matrix cores accumulate in FP32 over a short run of rows (32 in FP32,
// 128 in BF16), and each run's sums are then added into FP64 accumulators: a
// Gram summed in FP32 over a whole block moves the block's small singular
// subspaces by more than the FP32 mode allows, and the short FP32 runs keep
// that error well inside it.
// A work-group (8 waves) owns a 128 x 128 tile (ti <= tj) of G over one chunk
// of rows; wave (wr, wc) owns rows [32 wr, 32 wr + 32) and columns
// [64 wc, 64 wc + 64) of the tile: 2 x 4 blocks of 16 x 16.  The rows go
// through LDS in panels of 32; the next panel's global loads are in flight
// while the current one is multiplied.  Operand layouts (decoded on the GPU):
// lane l holds row l % 16 of A and column l % 16 of B, the same k for the same
// (lane, element) of A and B, and D(i, j) sits in register i % 4 of lane
// j + 16 (i / 4).
//   * BF16 panels are stored transposed, one word per pair of rows (even row
//     in the low half), 20 words per column, so that a lane reads its 8 rows
//     of one column with one 16-byte LDS read.  The 16-byte quads of a column
//     are swizzled by (column / 16) mod 4: writes are at most 2-way bank
//     conflicts and reads conflict-free.
//   * FP32 panels are row-major with 144 floats per row (reads conflict-free).
// Work-groups are dispatched to the 8 XCDs round-robin; the tile pairs of one
// chunk are given to work-groups of one XCD, so the chunk's rows are fetched
// into one L2 and read from there by all its tiles.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kLpRows = 32;        // rows per LDS panel
constexpr int kLpTWords = 20;      // words per column of a transposed bf16 panel (16 + pad)
constexpr int kXcdsGram = 8;

// 8 consecutive elements of one row, as loaded (16-byte words).
template <typename TA> struct Raw8 {
    static constexpr int N = (int)(8 * sizeof(TA) / 16);
    u32x4 w[N];
};

// Loads elements [col0, col0 + 8) of a row.  VEC: one to four 16-byte loads
// (the caller guarantees alignment and col0 + 8 <= c); otherwise element by
// element with the column clamped (masked when converted).
template <typename TA, bool VEC>
__device__ __forceinline__ void raw_load(const TA *__restrict__ rowp, int col0, int c, Raw8<TA> &r)
{
    if constexpr (VEC) {
        const u32x4 *p = reinterpret_cast<const u32x4 *>(rowp + col0);
#pragma unroll
        for (int i = 0; i < Raw8<TA>::N; ++i) r.w[i] = p[i];
    } else {
        TA v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = rowp[min(col0 + e, c - 1)];
        __builtin_memcpy(&r, v, sizeof v);
    }
}

__device__ __forceinline__ float raw_f32(const Raw8<uint16_t> &r, int e)
{
    return __uint_as_float(((r.w[0][e / 2] >> (16 * (e % 2))) & 0xFFFFu) << 16);
}
__device__ __forceinline__ float raw_f32(const Raw8<float> &r, int e) { return __uint_as_float(r.w[e / 4][e % 4]); }
__device__ __forceinline__ float raw_f32(const Raw8<double> &r, int e)
{
    const uint64_t u = ((uint64_t)r.w[e / 2][2 * (e % 2) + 1] << 32) | r.w[e / 2][2 * (e % 2)];
    return (float)__longlong_as_double((long long)u);
}

// bf16 bits rounded to nearest even from FP32 (finite values).
__device__ __forceinline__ uint32_t bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint32_t raw_bf16(const Raw8<uint16_t> &r, int e)
{
    return (r.w[0][e / 2] >> (16 * (e % 2))) & 0xFFFFu;
}
template <typename TA>
__device__ __forceinline__ uint32_t raw_bf16(const Raw8<TA> &r, int e) { return bf16_rne(raw_f32(r, e)); }

// TILE = 128: 8 waves of 32 x 64; TILE = 64: 4 waves of 32 x 32.  Every output
// element sees the same matrix-core operations in the same order in both (the
// same panels, the same FP32 runs), so the two compute the same bits.
template <int TILE, bool BF16, typename TA, bool VEC>
__global__ __launch_bounds__(TILE * 4) void gram_lp_kernel(const TA *__restrict__ X, int64_t ld, int c,
                                                             const Chunk *__restrict__ chunks, int nchunks,
                                                             int npairs, double *__restrict__ Gpart)
{
    // LDS: two strips (columns of tile ti and of tile tj) of one panel
    constexpr int FSTRIDE = TILE + 16;             // floats per row of an FP32 panel
    constexpr int CG = TILE / 8;                   // 8-column groups per strip
    constexpr int NBB = TILE / 32;                 // 16-column blocks per wave
    constexpr int BF_WORDS = 2 * TILE * kLpTWords;
    constexpr int F_WORDS = 2 * kLpRows * FSTRIDE;
    __shared__ __align__(16) uint32_t lds[BF16 ? BF_WORDS : F_WORDS];
    constexpr int FLUSH = BF16 ? 4 : 1;            // panels per FP32 run

    const int per = (nchunks + kXcdsGram - 1) / kXcdsGram;
    const int slot = (int)blockIdx.x / kXcdsGram;
    const int chunk = (int)(blockIdx.x % kXcdsGram) * per + slot / npairs;
    if (chunk >= nchunks) return;
    int idx = slot % npairs, ti = 0;
    const int ntile = (c + TILE - 1) / TILE;
    while (idx >= ntile - ti) { idx -= ntile - ti; ++ti; }
    const int tj = ti + idx;
    const bool diag = ti == tj;
    const Chunk ch = chunks[chunk];
    const TA *__restrict__ Xc = X + ch.x_off;
    const int rows = ch.rows;
    const int tid = threadIdx.x, lane = tid % 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int wr = wave / 2, wc = wave % 2;
    // 16 x 16 block (a, b) of this wave is block (2 wr + a, NBB wc + b) of the
    // tile; on a diagonal tile only blocks on or above the diagonal are formed
    const bool active = !(diag && 2 * wr > NBB * wc + NBB - 1) && ti * TILE + wr * 32 < c &&
                        tj * TILE + wc * 16 * NBB < c;

    // loads of a panel: BF16: thread -> strip, row pair bp (rows 2 bp,
    // 2 bp + 1) and 8-column group of that strip; FP32: thread -> row tid / CG
    // (0..31) and 8-column group tid % CG of both strips
    const int cg = tid % CG;
    constexpr int NR = 2;                          // raw items per thread
    Raw8<TA> ra[NR];
    const int bs = tid / (16 * CG), bp = (tid % (16 * CG)) / CG;
    auto item = [&](int h, int r0, int &row, int &col, int &s) {
        if constexpr (BF16) {
            s = bs;
            row = r0 + 2 * bp + h;
        } else {
            s = h;
            row = r0 + tid / CG;
        }
        col = (s == 0 ? ti : tj) * TILE + 8 * cg;
    };
    const bool loads = !(BF16 && diag && bs == 1);
    auto issue = [&](int r0) {
#pragma unroll
        for (int h = 0; h < NR; ++h) {
            int row, col, s;
            item(h, r0, row, col, s);
            if (!BF16 && diag && s == 1) continue;
            const int colc = VEC ? min(col, c - 8) : col;
            const int64_t rc = min(row, rows - 1);
            if (loads) raw_load<TA, VEC>(Xc + rc * ld, colc, c, ra[h]);
        }
    };
    auto stage = [&](int r0) {
        if constexpr (BF16) {
            if (!loads) return;
            int row, col, s;
            item(0, r0, row, col, s);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool cok = col + e < c;
                const uint32_t lo = (cok && row < rows) ? raw_bf16(ra[0], e) : 0u;
                const uint32_t hi = (cok && row + 1 < rows) ? raw_bf16(ra[1], e) : 0u;
                const int lc = 8 * cg + e;                     // column within the strip
                const int q = (bp >> 2) ^ ((lc >> 4) & 3);     // swizzled quad
                lds[(s * TILE + lc) * kLpTWords + 4 * q + (bp & 3)] = lo | (hi << 16);
            }
        } else {
#pragma unroll
            for (int h = 0; h < NR; ++h) {
                int row, col, s;
                item(h, r0, row, col, s);
                if (diag && s == 1) continue;
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = (row < rows && col + e < c) ? raw_f32(ra[h], e) : 0.0f;
                float *dst = reinterpret_cast<float *>(lds) + (s * kLpRows + tid / CG) * FSTRIDE + 8 * cg;
                *reinterpret_cast<v4f *>(dst) = (v4f){v[0], v[1], v[2], v[3]};
                *reinterpret_cast<v4f *>(dst + 4) = (v4f){v[4], v[5], v[6], v[7]};
            }
        }
    };

    v4f acc[2][NBB];
    double accd[2][NBB][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NBB; ++b) {
            acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) accd[a][b][v] = 0.0;
        }

    const int sj = diag ? 0 : 1;                   // strip of the B operand
    issue(0);
    int panel = 0;
    for (int r0 = 0; r0 < rows; r0 += kLpRows, ++panel) {
        __syncthreads();                           // the previous panel has been read
        stage(r0);
        __syncthreads();
        if (r0 + kLpRows < rows) issue(r0 + kLpRows);
        if (!active) continue;
        if constexpr (BF16) {
            v8bf fa[2], fb[NBB];
            const int g = lane / 16;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int ca = wr * 32 + 16 * a + lane % 16;
                fa[a] = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4 *>(
                    lds + ca * kLpTWords + 4 * (g ^ ((ca >> 4) & 3))));
            }
#pragma unroll
            for (int b = 0; b < NBB; ++b) {
                const int cb2 = wc * 16 * NBB + 16 * b + lane % 16;
                fb[b] = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4 *>(
                    lds + (sj * TILE + cb2) * kLpTWords + 4 * (g ^ ((cb2 >> 4) & 3))));
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < NBB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
        } else {
            const float *F = reinterpret_cast<const float *>(lds);
#pragma unroll 2
            for (int st = 0; st < kLpRows / 4; ++st) {
                const int rr = 4 * st + lane / 16;
                float fa[2], fb[NBB];
#pragma unroll
                for (int a = 0; a < 2; ++a) fa[a] = F[rr * FSTRIDE + wr * 32 + 16 * a + lane % 16];
#pragma unroll
                for (int b = 0; b < NBB; ++b)
                    fb[b] = F[(sj * kLpRows + rr) * FSTRIDE + wc * 16 * NBB + 16 * b + lane % 16];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < NBB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
            }
        }
        if ((panel + 1) % FLUSH == 0 || r0 + kLpRows >= rows) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < NBB; ++b) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) accd[a][b][v] += (double)acc[a][b][v];
                    acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
                }
        }
    }
    if (!active) return;
    // G(I, J) and its mirror; on a diagonal tile blocks below the diagonal are
    // skipped and diagonal blocks write i <= j only
    double *G = Gpart + (int64_t)ch.slot * c * c;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NBB; ++b) {
            const int A = 2 * wr + a, B = NBB * wc + b;
            if (diag && A > B) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * A + 4 * (lane / 16) + v, j = 16 * B + lane % 16;
                if (diag && A == B && i > j) continue;
                const int I = ti * TILE + i, J = tj * TILE + j;
                if (I < c && J < c) {
                    G[(int64_t)I * c + J] = accd[a][b][v];
                    G[(int64_t)J * c + I] = accd[a][b][v];
                }
            }
        }
}

template <int TILE, bool BF16, typename TA>
void run_gram_lp_t(const TA *X, int64_t ld, int c, const Chunk *chunks, int nchunks, double *Gpart,
                   hipStream_t stream)
{
    const int ntile = (c + TILE - 1) / TILE;
    const int npairs = ntile * (ntile + 1) / 2;
    const int per = (nchunks + kXcdsGram - 1) / kXcdsGram;
    const unsigned grid = (unsigned)(kXcdsGram * per * npairs);
    const bool vec = c % 8 == 0 && (ld * (int64_t)sizeof(TA)) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(X) % 16 == 0;
    if (vec)
        gram_lp_kernel<TILE, BF16, TA, true><<<grid, TILE * 4, 0, stream>>>(X, ld, c, chunks, nchunks,
                                                                           npairs, Gpart);
    else
        gram_lp_kernel<TILE, BF16, TA, false><<<grid, TILE * 4, 0, stream>>>(X, ld, c, chunks, nchunks,
                                                                            npairs, Gpart);
}

// Tile edge chosen by the autotuner (same bits either way).
template <bool BF16, typename TA>
hipError_t run_gram_lp(const TA *X, int64_t ld, int c, const Chunk *chunks, int nchunks, double *Gpart,
                       hipStream_t stream)
{
    char key[96];
    snprintf(key, sizeof key, "%s/%d c=%d n=%d", BF16 ? "bf16" : "f32", (int)sizeof(TA), c,
             tune_bucket(nchunks));
    return tuned_launch("gram_lp_tile", key, 2, 0, stream, [&](int v) {
        if (v == 0) run_gram_lp_t<128, BF16>(X, ld, c, chunks, nchunks, Gpart, stream);
        else run_gram_lp_t<64, BF16>(X, ld, c, chunks, nchunks, Gpart, stream);
        return hipGetLastError();
    });
}

template <typename TA>
void run_gram(const TA *X, int64_t ld, int c, const Chunk *chunks, int nchunks, double *Gpart,
              hipStream_t stream)
{
    // The matrix-core form for c <= 128.  Wider matrices need 16 block columns
    // of accumulators per wave, which leaves one wave per SIMD and exposes the
    // load latency (measured 3x slower than the register-tiled form at c = 256).
    if (c <= 128) {
        const int nb = (c + 15) / 16;
        const int waves = (nb + 1) / 2;            // two block columns per wave
        dim3 grid(nchunks, (waves + kThreads / 64 - 1) / (kThreads / 64));
        gram_mfma_kernel<8, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart);
        return;
    }
    const int tm = c <= 16 ? 1 : c <= 32 ? 2 : c <= 64 ? 4 : 8;
    const int tile = 16 * tm;
    const int ntile = (c + tile - 1) / tile;
    dim3 grid(nchunks, ntile * (ntile + 1) / 2);
    switch (tm) {
    case 1: gram_kernel<1, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart); break;
    case 2: gram_kernel<2, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart); break;
    case 4: gram_kernel<4, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart); break;
    default: gram_kernel<8, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart); break;
    }
}

hipError_t launch_gram(const void *X, int x_type, int64_t ld, int c, const Chunk *chunks,
                       int nchunks, double *Gpart, hipStream_t stream, int prec)
{
    if (nchunks <= 0) return hipSuccess;
    timing_begin("gram", stream);
    // bf16 input goes through the BF16 matrix cores in both reduced modes
    // (exact products); FP32 mode rounds wider input to FP32
    const bool bf = prec == kGramBF16 || (prec == kGramF32 && x_type == kElemBF16);
    if (prec != kGramF64) {
        hipError_t e;
        if (x_type == kElemBF16)
            e = run_gram_lp<true>(static_cast<const uint16_t *>(X), ld, c, chunks, nchunks, Gpart, stream);
        else if (x_type == kElemF32)
            e = bf ? run_gram_lp<true>(static_cast<const float *>(X), ld, c, chunks, nchunks, Gpart, stream)
                   : run_gram_lp<false>(static_cast<const float *>(X), ld, c, chunks, nchunks, Gpart, stream);
        else
            e = bf ? run_gram_lp<true>(static_cast<const double *>(X), ld, c, chunks, nchunks, Gpart, stream)
                   : run_gram_lp<false>(static_cast<const double *>(X), ld, c, chunks, nchunks, Gpart, stream);
        timing_end("gram", stream);
        return e;
    } else if (x_type == kElemF32)
        run_gram(static_cast<const float *>(X), ld, c, chunks, nchunks, Gpart, stream);
    else if (x_type == kElemBF16)
        run_gram(static_cast<const uint16_t *>(X), ld, c, chunks, nchunks, Gpart, stream);
    else
        run_gram(static_cast<const double *>(X), ld, c, chunks, nchunks, Gpart, stream);
    hipError_t e = hipGetLastError();
    timing_end("gram", stream);
    return e;
}

}  // namespace zs
