// Batched dense linear algebra kernels (FP64, MFMA 16x16x4 for the GEMM-shaped
// updates).  Every routine processes all items of a batch in one launch per
// algorithmic step; items of different sizes simply drop out of later steps.
#include "dense.hpp"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace dd {

// ===========================================================================
// GEMM
// ===========================================================================
template <bool TA, bool TB>
struct OpGemm {
    const GemmItem* g;
    __device__ int tiles(int b) const { return ceil_div_d(g[b].M, 64) * ceil_div_d(g[b].N, 64); }
    __device__ static int ceil_div_d(int a, int c) { return a > 0 ? (a + c - 1) / c : 0; }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemC sm;
        const GemmItem& G = g[b];
        const int tm = ceil_div_d(G.M, 64);
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        double4_t acc[2][2];
        acc_zero(acc);
        mfma_tile_64<TA, TB>(G.A, G.lda, G.B, G.ldb, G.M, G.N, G.K, i0, j0, sm.t, acc);
        double* C = G.C;
        const int ldc = G.ldc, M = G.M, N = G.N;
        const double al = G.alpha, be = G.beta;
        acc_store_coalesced(acc, sm, [&](int r, int c, double v) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < M && gj < N) {
                double* p = C + gi + (int64_t)gj * ldc;
                *p = (be == 0.0) ? al * v : al * v + be * *p;
            }
        });
    }
};

// The same on 128 x 128 tiles (mfma_tile_128), for batches of large products
template <bool TA, bool TB>
struct OpGemm128 {
    const GemmItem* g;
    __device__ int tiles(int b) const { return ((g[b].M + 127) / 128) * ((g[b].N + 127) / 128); }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmem128 sm;
        const GemmItem& G = g[b];
        if (G.M <= 0 || G.N <= 0) return;
        const int tm = (G.M + 127) / 128;
        const int i0 = (t % tm) * 128, j0 = (t / tm) * 128;
        Acc128 acc;
        acc128_zero(acc);
        mfma_tile_128<TA, TB>(G.A, G.lda, G.B, G.ldb, G.M, G.N, G.K, i0, j0, sm, acc);
        double* C = G.C;
        const int64_t ldc = G.ldc;
        const int M = G.M, N = G.N;
        const double al = G.alpha, be = G.beta;
        if (be == 0.0) {
            acc128_foreach(acc, [&](int r, int c, double v) {
                const int gi = i0 + r, gj = j0 + c;
                if (gi < M && gj < N) C[gi + (int64_t)gj * ldc] = al * v;
            });
        } else {
            acc128_axpby(acc, C, ldc, i0, j0, M, N, al, be);
        }
    }
};
template <bool TA, bool TB>
struct TileWaves<OpGemm128<TA, TB>> {
    static constexpr int value = 2;
};

// 128 x 128 tiles pay when the batch fills the GPU several times over with
// them and little of their area falls outside the matrices
static bool use_tile128(const std::vector<GemmItem>& items, bool lower_only) {
    double area = 0.0, padded = 0.0;
    int64_t t128 = 0;
    for (auto& x : items) {
        if (x.M <= 0 || x.N <= 0) continue;
        const int64_t a = ceil_div(x.M, 128), b = ceil_div(x.N, 128);
        const int64_t t = lower_only ? a * (a + 1) / 2 : a * b;
        t128 += t;
        padded += (double)t * 128.0 * 128.0;
        area += lower_only ? 0.5 * x.M * (x.M + 128.0) : (double)x.M * x.N;
    }
    return t128 >= 2048 && area >= 0.85 * padded;
}

void gemm_vb(Batch<GemmItem>& g, bool ta, bool tb, hipStream_t s) {
    if (use_tile128(g.h, false)) {
        int64_t total = 0;
        for (auto& x : g.h) total += (int64_t)ceil_div(x.M, 128) * ceil_div(x.N, 128);
        auto work = [&](int b0, int cnt, double& fl, double& by) {
            for (int i = b0; i < b0 + cnt; ++i) {
                const GemmItem& x = g.h[i];
                const double M = x.M, N = x.N, K = x.K;
                fl += 2.0 * M * N * K;
                by += 8.0 * (M * K + K * N + M * N * (x.beta != 0.0 ? 2.0 : 1.0));
            }
        };
        if (ta && tb) launch_tiles(OpGemm128<true, true>{g.d.p}, g.size(), total, s, "gemm_tt", 4096, work);
        else if (ta) launch_tiles(OpGemm128<true, false>{g.d.p}, g.size(), total, s, "gemm_tn", 4096, work);
        else if (tb) launch_tiles(OpGemm128<false, true>{g.d.p}, g.size(), total, s, "gemm_nt", 4096, work);
        else launch_tiles(OpGemm128<false, false>{g.d.p}, g.size(), total, s, "gemm_nn", 4096, work);
        return;
    }
    int64_t total = 0;
    for (auto& x : g.h) total += (int64_t)ceil_div(x.M, 64) * ceil_div(x.N, 64);
    // 2MNK flops; bytes = read A and B once, write C (and read it when beta != 0)
    auto work = [&](int b0, int cnt, double& fl, double& by) {
        for (int i = b0; i < b0 + cnt; ++i) {
            const GemmItem& x = g.h[i];
            const double M = x.M, N = x.N, K = x.K;
            fl += 2.0 * M * N * K;
            by += 8.0 * (M * K + K * N + M * N * (x.beta != 0.0 ? 2.0 : 1.0));
        }
    };
    if (ta && tb) launch_tiles(OpGemm<true, true>{g.d.p}, g.size(), total, s, "gemm_tt", 4096, work);
    else if (ta) launch_tiles(OpGemm<true, false>{g.d.p}, g.size(), total, s, "gemm_tn", 4096, work);
    else if (tb) launch_tiles(OpGemm<false, true>{g.d.p}, g.size(), total, s, "gemm_nt", 4096, work);
    else launch_tiles(OpGemm<false, false>{g.d.p}, g.size(), total, s, "gemm_nn", 4096, work);
}

// lower-triangle tiles (ti >= tj) of C = alpha A A^T + beta C
struct OpSyrk {
    const GemmItem* g;
    __device__ int tiles(int b) const {
        const int T = (g[b].M + 63) / 64;
        return T * (T + 1) / 2;
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemC sm;
        const GemmItem& G = g[b];
        int tj = 0, r = t;
        const int T = (G.M + 63) / 64;
        while (r >= T - tj) {
            r -= T - tj;
            ++tj;
        }
        const int ti = tj + r;
        const int i0 = ti * 64, j0 = tj * 64;
        double4_t acc[2][2];
        acc_zero(acc);
        mfma_tile_64<false, true>(G.A, G.lda, G.A, G.lda, G.M, G.M, G.K, i0, j0, sm.t, acc);
        double* C = G.C;
        const int ldc = G.ldc, M = G.M;
        const double al = G.alpha, be = G.beta;
        acc_store_coalesced(acc, sm, [&](int rr, int c, double v) {
            const int gi = i0 + rr, gj = j0 + c;
            if (gi < M && gj < M) {
                double* p = C + gi + (int64_t)gj * ldc;
                *p = (be == 0.0) ? al * v : al * v + be * *p;
            }
        });
    }
};
// The same on 128 x 128 tiles
struct OpSyrk128 {
    const GemmItem* g;
    __device__ int tiles(int b) const {
        const int T = (g[b].M + 127) / 128;
        return T * (T + 1) / 2;
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmem128 sm;
        const GemmItem& G = g[b];
        if (G.M <= 0) return;
        int tj = 0, r = t;
        const int T = (G.M + 127) / 128;
        while (r >= T - tj) {
            r -= T - tj;
            ++tj;
        }
        const int ti = tj + r;
        const int i0 = ti * 128, j0 = tj * 128;
        Acc128 acc;
        acc128_zero(acc);
        mfma_tile_128<false, true>(G.A, G.lda, G.A, G.lda, G.M, G.M, G.K, i0, j0, sm, acc);
        double* C = G.C;
        const int64_t ldc = G.ldc;
        const int M = G.M;
        const double al = G.alpha, be = G.beta;
        if (be == 0.0) {
            acc128_foreach(acc, [&](int rr, int c, double v) {
                const int gi = i0 + rr, gj = j0 + c;
                if (gi < M && gj < M) C[gi + (int64_t)gj * ldc] = al * v;
            });
        } else {
            acc128_axpby(acc, C, ldc, i0, j0, M, M, al, be);
        }
    }
};
template <>
struct TileWaves<OpSyrk128> {
    static constexpr int value = 2;
};

void syrk_vb(Batch<GemmItem>& g, hipStream_t s) {
    if (use_tile128(g.h, true)) {
        int64_t total = 0;
        for (auto& x : g.h) {
            const int64_t T = ceil_div(x.M, 128);
            total += T * (T + 1) / 2;
        }
        launch_tiles(OpSyrk128{g.d.p}, g.size(), total, s, "syrk");
        return;
    }
    int64_t total = 0;
    for (auto& x : g.h) {
        const int64_t T = ceil_div(x.M, 64);
        total += T * (T + 1) / 2;
    }
    launch_tiles(OpSyrk{g.d.p}, g.size(), total, s, "syrk");
}

// C = alpha A B + beta C, A upper triangular: row tile i0 only needs k >= i0
struct OpGemmUpperA {
    const GemmItem* g;
    __device__ int tiles(int b) const { return ((g[b].M + 63) / 64) * ((g[b].N + 63) / 64); }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemC sm;
        const GemmItem& G = g[b];
        const int tm = (G.M + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        double4_t acc[2][2];
        acc_zero(acc);
        mfma_tile_64<false, false>(G.A + (int64_t)i0 * G.lda, G.lda, G.B + i0, G.ldb, G.M, G.N, G.K - i0, i0, j0, sm.t, acc);
        double* C = G.C;
        const int ldc = G.ldc, M = G.M, N = G.N;
        const double al = G.alpha, be = G.beta;
        acc_store_coalesced(acc, sm, [&](int r, int c, double v) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < M && gj < N) {
                double* p = C + gi + (int64_t)gj * ldc;
                *p = (be == 0.0) ? al * v : al * v + be * *p;
            }
        });
    }
};
void gemm_upper_a_vb(Batch<GemmItem>& g, hipStream_t s) {
    int64_t total = 0;
    for (auto& x : g.h) total += (int64_t)ceil_div(x.M, 64) * ceil_div(x.N, 64);
    launch_tiles(OpGemmUpperA{g.d.p}, g.size(), total, s, "gemm_upper_a");
}

// ===========================================================================
// x := W^T (W x), W lower triangular (explicit inverse of a Cholesky factor).
// HBM-bound: each pass streams the lower triangle of W once.
// ===========================================================================
// y_part[cc] = W(rb rows, cc columns) x(cc columns): a tile is a 64-row block
// by a 512-column chunk; lane = row (coalesced 512 B column segments), wave w
// takes columns w, w+4, ... of the chunk.  Chunks right of the block's
// diagonal are skipped (W is zero there).
template <class TW>
struct OpTrmvN {
    const TrmvItemT<TW>* it;
    __device__ static int nrb(int n) { return (n + TRMV_RB - 1) / TRMV_RB; }
    __device__ static int ncc(int n) { return (n + TRMV_CC - 1) / TRMV_CC; }
    __device__ int tiles(int b) const { return nrb(it[b].n) * ncc(it[b].n); }
    __device__ void operator()(int b, int t) const {
        __shared__ double red[4][TRMV_RB];
        const TrmvItemT<TW>& I = it[b];
        const int n = I.n, nc = ncc(n);
        const int rb = t / nc, cc = t % nc;
        const int r0 = rb * TRMV_RB, c0 = cc * TRMV_CC;
        if (c0 > r0 + TRMV_RB - 1) return;  // above the diagonal: no partial (reducer skips it)
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int r = r0 + lane;
        const int cend = min(min(c0 + TRMV_CC, n), r0 + TRMV_RB);
        TW a0 = 0, a1 = 0, a2 = 0, a3 = 0;  // arithmetic in the factor's precision
        if (r < n) {
            const TW* Wr = I.W + r;
            int j = c0 + w;
            for (; j + 12 < cend; j += 16) {
                a0 += Wr[(int64_t)j * I.ld] * (TW)I.x[j];
                a1 += Wr[(int64_t)(j + 4) * I.ld] * (TW)I.x[j + 4];
                a2 += Wr[(int64_t)(j + 8) * I.ld] * (TW)I.x[j + 8];
                a3 += Wr[(int64_t)(j + 12) * I.ld] * (TW)I.x[j + 12];
            }
            for (; j < cend; j += 4) a0 += Wr[(int64_t)j * I.ld] * (TW)I.x[j];
        }
        red[w][lane] = (double)((a0 + a1) + (a2 + a3));
        __syncthreads();
        if (w == 0 && r < n)
            I.part[(int64_t)cc * n + r] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    }
};
// y = sum of the partials of the chunks left of (or at) the row's block diagonal
template <class TW>
struct OpTrmvRed {
    const TrmvItemT<TW>* it;
    __device__ int tiles(int b) const { return (it[b].n + 255) / 256; }
    __device__ void operator()(int b, int t) const {
        const TrmvItemT<TW>& I = it[b];
        const int r = t * 256 + threadIdx.x;
        if (r >= I.n) return;
        const int last = ((r / TRMV_RB) * TRMV_RB + TRMV_RB - 1) / TRMV_CC;
        double v = 0.0;
        for (int cc = 0; cc <= last; ++cc) v += I.part[(int64_t)cc * I.n + r];
        I.y[r] = v;
    }
};
// x_j = W(j:n, j)^T y(j:n): a tile is 16 columns (4 per wave, each a
// contiguous column segment read by the 64 lanes) by a chunk of TRMV_CC rows
// at or below the columns' diagonal block; its dots go to part[chunk n + j]
// and OpTrmvTRed sums them.  Short chunks keep every wave's chain of
// dependent loads short.
template <class TW>
struct OpTrmvT {
    const TrmvItemT<TW>* it;
    __device__ int tiles(int b) const { return trmv_t_tiles(it[b].n); }
    __device__ void operator()(int b, int t) const {
        const TrmvItemT<TW>& I = it[b];
        const int n = I.n;
        const int ng = (n + 15) / 16;
        int c = 0, g = t;
        for (;;) {
            const int k = min(ng, (TRMV_CC / 16) * (c + 1));
            if (g < k) break;
            g -= k;
            ++c;
        }
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int j0 = g * 16 + w * 4;
        const int rb = max(c * TRMV_CC, g * 16), re = min(n, (c + 1) * TRMV_CC);
        TW accw[4] = {0, 0, 0, 0};
        if (j0 < n) {
            const int jn = min(4, n - j0);
            // W is zero above the diagonal, so rows from the block's first column on
            for (int i = rb + lane; i < re; i += 64) {
                const TW yi = (TW)I.y[i];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q < jn) accw[q] += I.W[i + (int64_t)(j0 + q) * I.ld] * yi;
            }
        }
        double acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = wave_sum((double)accw[q]);
        if (lane == 0)
            for (int q = 0; q < 4; ++q)
                if (j0 + q < n) I.part[(int64_t)c * n + j0 + q] = acc[q];
    }
};
// x_j = sum of the partials of the chunks from the one holding j on
template <class TW>
struct OpTrmvTRed {
    const TrmvItemT<TW>* it;
    __device__ int tiles(int b) const { return (it[b].n + 255) / 256; }
    __device__ void operator()(int b, int t) const {
        const TrmvItemT<TW>& I = it[b];
        const int j = t * 256 + threadIdx.x;
        if (j >= I.n) return;
        const int nch = (I.n + TRMV_CC - 1) / TRMV_CC;
        double v = 0.0;
        for (int c = j / TRMV_CC; c < nch; ++c) v += I.part[(int64_t)c * I.n + j];
        I.x[j] = v;
    }
};

template <class TW>
static void trmv_n_t(Batch<TrmvItemT<TW>>& t, hipStream_t s) {
    int64_t tn = 0, tr = 0;
    for (auto& x : t.h) {
        tn += (int64_t)ceil_div(x.n, TRMV_RB) * ceil_div(x.n, TRMV_CC);
        tr += ceil_div(x.n, 256);
    }
    launch_tiles(OpTrmvN<TW>{t.d.p}, t.size(), tn, s, "trmv_n");
    launch_tiles(OpTrmvRed<TW>{t.d.p}, t.size(), tr, s, "trmv_red");
}
template <class TW>
static void trmv_t_t(Batch<TrmvItemT<TW>>& t, hipStream_t s) {
    int64_t tt = 0, tr = 0;
    for (auto& x : t.h) {
        tt += trmv_t_tiles(x.n);
        tr += ceil_div(x.n, 256);
    }
    launch_tiles(OpTrmvT<TW>{t.d.p}, t.size(), tt, s, "trmv_t");
    launch_tiles(OpTrmvTRed<TW>{t.d.p}, t.size(), tr, s, "trmv_t_red");
}

void trmv_n_vb(Batch<TrmvItem>& t, hipStream_t s) { trmv_n_t(t, s); }
void trmv_t_vb(Batch<TrmvItem>& t, hipStream_t s) { trmv_t_t(t, s); }
void trinv_apply_vb(Batch<TrmvItem>& t, hipStream_t s) {
    trmv_n_t(t, s);
    trmv_t_t(t, s);
}
void trinv_apply_vb(Batch<TrmvItem32>& t, hipStream_t s) {
    trmv_n_t(t, s);
    trmv_t_t(t, s);
}

// column sums: a wave per column (contiguous); row sums: a thread per row,
// columns in order (coalesced across the rows of a 256-row tile)
struct OpAbsCol {
    const DMat* A;
    double* const* out;
    __device__ int tiles(int b) const { return (A[b].n + 15) / 16; }
    __device__ void operator()(int b, int t) const {
        const DMat M = A[b];
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        for (int q = 0; q < 4; ++q) {
            const int c = t * 16 + w * 4 + q;
            if (c >= M.n) break;
            double s = 0.0;
            for (int r = lane; r < M.m; r += 64) s += fabs(M.p[r + (int64_t)c * M.ld]);
            s = wave_sum(s);
            if (lane == 0) out[b][c] = s;
        }
    }
};
struct OpAbsRow {
    const DMat* A;
    double* const* out;
    __device__ int tiles(int b) const { return (A[b].m + 255) / 256; }
    __device__ void operator()(int b, int t) const {
        const DMat M = A[b];
        const int r = t * 256 + threadIdx.x;
        if (r >= M.m) return;
        double s = 0.0;
        for (int c = 0; c < M.n; ++c) s += fabs(M.p[r + (int64_t)c * M.ld]);
        out[b][r] = s;
    }
};
void abs_sums_vb(Batch<DMat>& A, double* const* colsum, double* const* rowsum, hipStream_t s) {
    int64_t tc = 0, tr = 0;
    for (auto& x : A.h) {
        tc += ceil_div(x.n, 16);
        tr += ceil_div(x.m, 256);
    }
    launch_tiles(OpAbsCol{A.d.p, colsum}, A.size(), tc, s, "abs_col");
    launch_tiles(OpAbsRow{A.d.p, rowsum}, A.size(), tr, s, "abs_row");
}

__global__ void k_to_fp32(const double* src, float* dst, int64_t n, int* bad) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = (float)src[i];
        dst[i] = v;
        if (!isfinite(v)) *bad = 1;  // every writer stores the same value
    }
}
void to_fp32(const double* src, float* dst, int64_t n, int* bad, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_fp32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s, src, dst,
                       n, bad);
    launch_check("to_fp32");
}

// ===========================================================================
// FP32 local factors: Jacobi scaling, identity, column scaling (one column of
// one item per tile, 256 rows per pass)
// ===========================================================================
struct OpJacobiDiag {
    const Fp32Item* f;
    __device__ int tiles(int b) const { return (f[b].n + 255) / 256; }
    __device__ void operator()(int b, int t) const {
        const Fp32Item& it = f[b];
        const int k = t * 256 + (int)threadIdx.x;
        if (k < it.n) {
            const double a = it.A[k + (int64_t)k * it.n];
            it.d[k] = a > 0.0 ? 1.0 / sqrt(a) : 1.0;
        }
    }
};
struct OpJacobiScale {
    const Fp32Item* f;
    __device__ int tiles(int b) const { return f[b].n; }
    __device__ void operator()(int b, int c) const {
        const Fp32Item& it = f[b];
        const int n = it.n;
        const double dc = it.d[c];
        const double* a = it.A + (int64_t)c * n;
        float* o = it.A32 + (int64_t)c * n;
        for (int r = threadIdx.x; r < n; r += blockDim.x) o[r] = r >= c ? (float)(a[r] * it.d[r] * dc) : 0.0f;
    }
};
struct OpIdentity32 {
    const Fp32Item* f;
    __device__ int tiles(int b) const { return f[b].n; }
    __device__ void operator()(int b, int c) const {
        const Fp32Item& it = f[b];
        float* o = it.W32 + (int64_t)c * it.n;
        for (int r = threadIdx.x; r < it.n; r += blockDim.x) o[r] = r == c ? 1.0f : 0.0f;
    }
};
struct OpScaleCols32 {
    const Fp32Item* f;
    __device__ int tiles(int b) const { return f[b].n; }
    __device__ void operator()(int b, int c) const {
        const Fp32Item& it = f[b];
        const float dc = (float)it.d[c];
        float* o = it.W32 + (int64_t)c * it.n;
        bool fin = true;
        for (int r = c + threadIdx.x; r < it.n; r += blockDim.x) {
            const float v = o[r] * dc;
            o[r] = v;
            fin = fin && isfinite(v);
        }
        if (!fin) *it.bad = 1;  // every writer stores the same value
    }
};
template <bool TO32>
struct OpRowScale {
    const RowScaleItem* r;
    __device__ int tiles(int b) const { return r[b].k; }
    __device__ void operator()(int b, int c) const {
        const RowScaleItem& it = r[b];
        double* B = it.B + (int64_t)c * it.n;
        float* B32 = it.B32 + (int64_t)c * it.n;
        for (int i = threadIdx.x; i < it.n; i += blockDim.x) {
            if (TO32) B32[i] = (float)(it.d[i] * B[i]);
            else B[i] = it.d[i] * (double)B32[i];
        }
    }
};
void rowscale_fp32_vb(Batch<RowScaleItem>& r, bool to32, hipStream_t s) {
    int64_t nc = 0;
    for (auto& x : r.h) nc += x.k;
    if (!nc) return;
    if (to32) launch_tiles(OpRowScale<true>{r.d.p}, r.size(), nc, s, "rowscale_to32");
    else launch_tiles(OpRowScale<false>{r.d.p}, r.size(), nc, s, "rowscale_from32");
}
void jacobi_fp32_vb(Batch<Fp32Item>& f, hipStream_t s) {
    int64_t nd = 0, nc = 0;
    for (auto& x : f.h) {
        nd += ceil_div(x.n, 256);
        nc += x.n;
    }
    launch_tiles(OpJacobiDiag{f.d.p}, f.size(), nd, s, "jacobi_diag");
    launch_tiles(OpJacobiScale{f.d.p}, f.size(), nc, s, "jacobi_fp32");
}
void identity_fp32_vb(Batch<Fp32Item>& f, hipStream_t s) {
    int64_t nc = 0;
    for (auto& x : f.h) nc += x.n;
    launch_tiles(OpIdentity32{f.d.p}, f.size(), nc, s, "identity_fp32");
}
void scale_cols_fp32_vb(Batch<Fp32Item>& f, hipStream_t s) {
    int64_t nc = 0;
    for (auto& x : f.h) nc += x.n;
    launch_tiles(OpScaleCols32{f.d.p}, f.size(), nc, s, "scale_cols_fp32");
}

// ===========================================================================
// Cholesky (right-looking, 64-column blocks)
// Cholesky of the 64 x 64 diagonal block at k0 by one wave: lane i holds
// row i in registers; column j's pivot and entries reach the other lanes by
// cross-lane shuffles, so no step waits on a workgroup barrier.  A
// pivot not above piv_min (0 in FP64) records info = its 1-based column and
// continues with 1.  T = double or float (the FP32 local factors).
template <class T>
struct OpPotrfDiag {
    const MatT<T>* A;
    int* info;
    int k0;
    T piv_min;
    __device__ int tiles(int b) const { return A[b].n > k0 ? 1 : 0; }
    __device__ void operator()(int b, int) const {
        if (threadIdx.x >= 64) return;  // one wave; no workgroup barrier below
        const MatT<T> M = A[b];
        const int w = min(64, M.n - k0);
        const int64_t ld = M.ld;
        T* base = M.p + k0 + (int64_t)k0 * ld;
        const int i = threadIdx.x;
        T a[64];
#pragma unroll
        for (int c = 0; c < 64; ++c) a[c] = (i < w && c < w && i >= c) ? base[i + c * ld] : T(0);
        int bad = 0;
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            if (j < w) {
                T d = readlane_t(a[j], j);
                if (!(d > piv_min)) {
                    if (!bad) bad = j + 1;
                    d = T(1);
                }
                const T piv = sqrt(d);
                const T l = (i > j) ? a[j] / piv : (i == j ? piv : T(0));
                if (i < w && i >= j) base[i + j * ld] = l;  // column j is final
#pragma unroll
                for (int c = j + 1; c < 64; ++c) {
                    const T lc = readlane_t(l, c);
                    if (i >= c) a[c] -= l * lc;
                }
            }
        }
        if (bad && i == 0 && info[b] == 0) info[b] = k0 + bad;
    }
};

// A21 := A21 L11^{-T} for the rows below the diagonal block (down to m) by
// forward substitution, one row per thread, 256 rows per workgroup.
template <class T>
struct OpPotrfPanel {
    const MatT<T>* A;
    int k0;
    __device__ int tiles(int b) const {
        if (A[b].n <= k0) return 0;
        const int w = min(64, A[b].n - k0);
        const int rem = A[b].m - k0 - w;
        return rem > 0 ? (rem + 255) / 256 : 0;
    }
    __device__ void operator()(int b, int t) const {
        __shared__ T L[64][65];
        const MatT<T> M = A[b];
        const int w = min(64, M.n - k0);
        T* base = M.p + k0 + (int64_t)k0 * M.ld;
        for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
            const int r = e & 63, c = e >> 6;
            L[r][c] = (r < w && c < w && r >= c) ? base[r + (int64_t)c * M.ld] : T(0);
        }
        __syncthreads();
        const int row = k0 + w + t * 256 + (int)threadIdx.x;
        if (row < M.m) {
            T x[64];
            T* a = M.p + row + (int64_t)k0 * M.ld;
#pragma unroll
            for (int j = 0; j < 64; ++j) x[j] = (j < w) ? a[(int64_t)j * M.ld] : T(0);
#pragma unroll
            for (int j = 0; j < 64; ++j) {
                if (j < w) {
                    T v = x[j];
#pragma unroll
                    for (int l = 0; l < j; ++l) v -= x[l] * L[j][l];
                    x[j] = v / L[j][j];
                }
            }
#pragma unroll
            for (int j = 0; j < 64; ++j)
                if (j < w) a[(int64_t)j * M.ld] = x[j];
        }
    }
};

// Left-looking block update of the recursion: columns [mid, c1) and rows
// [mid, m) take -= A[mid:m, c0:mid] A[mid:c1, c0:mid]^T (lower part only
// inside the square block).
template <class T>
struct OpPotrfUpdate {
    const MatT<T>* A;
    int c0, mid, c1;
    __device__ void dims(const MatT<T>& M, int& TR, int& TC) const {
        const int rows = M.m - mid, cols = min(c1, M.n) - mid;
        TR = rows > 0 ? (rows + 63) / 64 : 0;
        TC = cols > 0 ? (cols + 63) / 64 : 0;
    }
    __device__ int tiles(int b) const {
        if (A[b].n <= mid) return 0;
        int TR, TC;
        dims(A[b], TR, TC);
        return TC * TR - TC * (TC - 1) / 2;
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemCT<T> sm;
        const MatT<T> M = A[b];
        int TR, TC;
        dims(M, TR, TC);
        int tj = 0, rem_t = t;
        while (rem_t >= TR - tj) {
            rem_t -= TR - tj;
            ++tj;
        }
        const int ti = tj + rem_t;
        const int rows = M.m - mid, cols = min(c1, M.n) - mid;
        const T* A21 = M.p + mid + (int64_t)c0 * M.ld;
        typename Vec4<T>::type acc[2][2];
        acc_zero(acc);
        mfma_tile_64<false, true>(A21, M.ld, A21, M.ld, rows, cols, mid - c0, ti * 64, tj * 64, sm.t, acc);
        T* C = M.p + mid + (int64_t)mid * M.ld;
        acc_store_coalesced(acc, sm, [&](int r, int c, T v) {
            const int gi = ti * 64 + r, gj = tj * 64 + c;
            if (gi < rows && gj < cols && gi >= gj) C[gi + (int64_t)gj * M.ld] -= v;
        });
    }
};

// Recursive (left half, update, right half) Cholesky of columns [c0, c1).
template <class T>
static const char* fp_name(const char* f64, const char* f32) {
    return std::is_same<T, float>::value ? f32 : f64;
}

template <class T>
static void potrf_rec(Batch<MatT<T>>& A, int* dinfo, T piv_min, int c0, int c1, hipStream_t s) {
    if (c1 - c0 <= 64) {
        int64_t nd = 0, np = 0;
        for (auto& x : A.h) {
            if (x.n <= c0) continue;
            ++nd;
            const int rem = x.m - c0 - std::min(64, x.n - c0);
            if (rem > 0) np += ceil_div(rem, 256);
        }
        if (!nd) return;
        launch_tiles(OpPotrfDiag<T>{A.d.p, dinfo, c0, piv_min}, A.size(), nd, s, fp_name<T>("potrf_diag", "potrf32_diag"));
        if (np) launch_tiles(OpPotrfPanel<T>{A.d.p, c0}, A.size(), np, s, fp_name<T>("potrf_panel", "potrf32_panel"));
        return;
    }
    const int mid = c0 + ceil_div(c1 - c0, 128) * 64;
    potrf_rec(A, dinfo, piv_min, c0, mid, s);
    int64_t nu = 0;
    for (auto& x : A.h) {
        if (x.n <= mid) continue;
        const int TR = ceil_div(x.m - mid, 64), TC = ceil_div(std::min(c1, x.n) - mid, 64);
        nu += (int64_t)TC * TR - (int64_t)TC * (TC - 1) / 2;
    }
    if (nu) launch_tiles(OpPotrfUpdate<T>{A.d.p, c0, mid, c1}, A.size(), nu, s, fp_name<T>("potrf_update", "potrf32_update"));
    potrf_rec(A, dinfo, piv_min, mid, c1, s);
}

void potrf_vb(Batch<DMat>& A, int* dinfo, hipStream_t s) {
    int nmax = 0;
    for (auto& x : A.h) nmax = std::max(nmax, x.n);
    if (nmax == 0) return;
    potrf_rec(A, dinfo, 0.0, 0, ceil_div(nmax, 64) * 64, s);
}
void potrf_vb(Batch<FMat>& A, int* dinfo, float piv_min, hipStream_t s) {
    int nmax = 0;
    for (auto& x : A.h) nmax = std::max(nmax, x.n);
    if (nmax == 0) return;
    potrf_rec(A, dinfo, piv_min, 0, ceil_div(nmax, 64) * 64, s);
}

// ===========================================================================
// Triangular solves with a lower factor, many right-hand sides
// ===========================================================================
// Inverses of the 64 x 64 diagonal blocks of L (lower): block t of item b
// goes to D[b] + 4096 t (column-major, ld 64), padded with the identity past
// the matrix edge.  Forward substitution on the identity, 4 threads per
// column sharing each dot product.
template <class T>
struct OpTrtri64 {
    const MatT<T>* L;
    T* const* D;
    __device__ int tiles(int b) const { return (L[b].n + 63) / 64; }
    __device__ void operator()(int b, int t) const {
        __shared__ T Ls[64][65];
        __shared__ T X[64][65];
        __shared__ T red[4][64];
        const MatT<T> Lm = L[b];
        const int k0 = t * 64, w = min(64, Lm.n - k0);
        const T* lb = Lm.p + k0 + (int64_t)k0 * Lm.ld;
        for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
            const int r = e & 63, c = e >> 6;
            T v = T(0);
            if (r >= c) v = (r < w) ? lb[r + (int64_t)c * Lm.ld] : (r == c ? T(1) : T(0));
            Ls[r][c] = v;
            X[r][c] = T(0);
        }
        __syncthreads();
        const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
        for (int i = 0; i < 64; ++i) {
            T sum = T(0);
            for (int l = q; l < i; l += 4) sum += Ls[i][l] * X[l][c];
            red[q][c] = sum;
            __syncthreads();
            if (q == 0) X[i][c] = ((i == c ? T(1) : T(0)) - ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c]))) / Ls[i][i];
            __syncthreads();
        }
        T* out = D[b] + (int64_t)t * 4096;
        for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) out[e] = X[e & 63][e >> 6];
    }
};

// Diagonal step: B[kb:kb+w, cols] := L_kk^{-1} B (or L_kk^{-T} B) as an MFMA
// product with the precomputed inverse; each tile owns 64 right-hand-side
// columns and reads them completely before writing them back.
template <class T, bool TRANS>
struct OpTrsmDiag {
    const MatT<T>* L;
    const MatT<T>* B;
    T* const* D;
    int kb;   // first row of the diagonal block
    int ncap; // column tiles that can be nonzero (lower-triangular right-hand side), or a large value
    __device__ int tiles(int b) const { return (L[b].n > kb) ? min((B[b].n + 63) / 64, ncap) : 0; }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemCT<T> sm;
        const MatT<T> Lm = L[b], Bm = B[b];
        const int w = min(64, Lm.n - kb);
        const int c0 = t * 64;
        const T* Di = D[b] + (int64_t)(kb / 64) * 4096;
        T* bb = Bm.p + kb;
        typename Vec4<T>::type acc[2][2];
        acc_zero(acc);
        mfma_tile_64<TRANS, false>(Di, 64, (const T*)bb, Bm.ld, w, Bm.n, w, 0, c0, sm.t, acc);
        const int ld = Bm.ld, N = Bm.n;
        acc_store_coalesced(acc, sm, [&](int r, int c, T v) {
            const int gj = c0 + c;
            if (r < w && gj < N) bb[r + (int64_t)gj * ld] = v;
        });
    }
};

// Recursive update of a triangular solve over rows [r0, r1) split at mid:
// forward  B[mid:e, :] -= L[mid:e, r0:mid] B[r0:mid, :]
// backward B[r0:mid, :] -= L[mid:e, r0:mid]^T B[mid:e, :],  e = min(n, r1)
template <class T, bool TRANS>
struct OpTrsmGemm {
    const MatT<T>* L;
    const MatT<T>* B;
    int r0, mid, r1;
    int ncap;  // column tiles that can be nonzero (lower-triangular right-hand side), or a large value
    __device__ int tiles(int b) const {
        const int n = L[b].n;
        if (n <= mid) return 0;
        const int e = min(n, r1);
        const int M = TRANS ? mid - r0 : e - mid;
        return ((M + 63) / 64) * min((B[b].n + 63) / 64, ncap);
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemCT<T> sm;
        const MatT<T> Lm = L[b], Bm = B[b];
        const int e = min(Lm.n, r1);
        const int M = TRANS ? mid - r0 : e - mid;
        const int K = TRANS ? e - mid : mid - r0;
        const int tm = (M + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        typename Vec4<T>::type acc[2][2];
        acc_zero(acc);
        const T* A = Lm.p + mid + (int64_t)r0 * Lm.ld;  // L[mid:e, r0:mid]
        T* Cp;
        if (!TRANS) {
            mfma_tile_64<false, false>(A, Lm.ld, (const T*)(Bm.p + r0), Bm.ld, M, Bm.n, K, i0, j0, sm.t, acc);
            Cp = Bm.p + mid;
        } else {
            mfma_tile_64<true, false>(A, Lm.ld, (const T*)(Bm.p + mid), Bm.ld, M, Bm.n, K, i0, j0, sm.t, acc);
            Cp = Bm.p + r0;
        }
        const int N = Bm.n, ld = Bm.ld;
        acc_store_coalesced(acc, sm, [&](int r, int c, T v) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < M && gj < N) Cp[gi + (int64_t)gj * ld] -= v;
        });
    }
};

// lower_rhs (forward solves only): B is lower triangular on entry (e.g. the
// identity), so column j stays zero in rows < j and column tiles right of the
// rows being solved are skipped.
template <class T>
static void trsm_rec(Batch<MatT<T>>& L, Batch<MatT<T>>& B, T* const* D, bool trans, bool lower_rhs, int r0, int r1,
                     hipStream_t s) {
    constexpr int kAll = 1 << 30;
    if (r1 - r0 <= 64) {
        const int cap = lower_rhs ? r0 / 64 + 1 : kAll;
        int64_t nd = 0;
        for (int b = 0; b < L.size(); ++b)
            if (L.h[b].n > r0) nd += std::min(ceil_div(B.h[b].n, 64), cap);
        if (!nd) return;
        if (!trans) launch_tiles(OpTrsmDiag<T, false>{L.d.p, B.d.p, D, r0, cap}, L.size(), nd, s, fp_name<T>("trsm_diag", "trsm32_diag"));
        else launch_tiles(OpTrsmDiag<T, true>{L.d.p, B.d.p, D, r0, cap}, L.size(), nd, s, fp_name<T>("trsmT_diag", "trsm32T_diag"));
        return;
    }
    const int mid = r0 + ceil_div(r1 - r0, 128) * 64;
    const int cap = lower_rhs ? mid / 64 : kAll;
    int64_t nu = 0;
    for (int b = 0; b < L.size(); ++b) {
        const int n = L.h[b].n;
        if (n <= mid) continue;
        const int e = std::min(n, r1);
        const int M = trans ? mid - r0 : e - mid;
        nu += (int64_t)ceil_div(M, 64) * std::min(ceil_div(B.h[b].n, 64), cap);
    }
    if (!trans) {
        trsm_rec(L, B, D, trans, lower_rhs, r0, mid, s);
        if (nu) launch_tiles(OpTrsmGemm<T, false>{L.d.p, B.d.p, r0, mid, r1, cap}, L.size(), nu, s, fp_name<T>("trsm_gemm", "trsm32_gemm"));
        trsm_rec(L, B, D, trans, lower_rhs, mid, r1, s);
    } else {
        trsm_rec(L, B, D, trans, lower_rhs, mid, r1, s);
        if (nu) launch_tiles(OpTrsmGemm<T, true>{L.d.p, B.d.p, r0, mid, r1, cap}, L.size(), nu, s, fp_name<T>("trsmT_gemm", "trsm32T_gemm"));
        trsm_rec(L, B, D, trans, lower_rhs, r0, mid, s);
    }
}

template <class T>
static void trsm_any(Batch<MatT<T>>& L, Batch<MatT<T>>& B, bool trans, hipStream_t s, bool lower_rhs) {
    int nmax = 0;
    for (auto& x : L.h) nmax = std::max(nmax, x.n);
    if (nmax == 0) return;
    // inverses of the 64 x 64 diagonal blocks
    std::vector<int64_t> off(L.size() + 1, 0);
    int64_t nblk = 0;
    for (int b = 0; b < L.size(); ++b) {
        const int k = ceil_div(L.h[b].n, 64);
        off[b + 1] = off[b] + (int64_t)k * 4096;
        nblk += k;
    }
    DBuf<T> dbuf(std::max<int64_t>(1, off.back()));
    std::vector<T*> hp(L.size());
    for (int b = 0; b < L.size(); ++b) hp[b] = dbuf.p + off[b];
    DBuf<T*> dp(std::max<size_t>(1, hp.size()));
    h2d(dp.p, hp.data(), hp.size(), s);
    launch_tiles(OpTrtri64<T>{L.d.p, dp.p}, L.size(), nblk, s, fp_name<T>("trtri64", "trtri64_32"));
    trsm_rec(L, B, dp.p, trans, lower_rhs && !trans, 0, ceil_div(nmax, 64) * 64, s);
    DD_HIP(hipStreamSynchronize(s));  // dbuf, dp are freed on return
}
void trsm_vb(Batch<DMat>& L, Batch<DMat>& B, bool trans, hipStream_t s, bool lower_rhs) {
    trsm_any(L, B, trans, s, lower_rhs);
}
void trsm_vb(Batch<FMat>& L, Batch<FMat>& B, bool trans, hipStream_t s, bool lower_rhs) {
    trsm_any(L, B, trans, s, lower_rhs);
}

// ===========================================================================
// Householder QR (32-column panels, compact WY)
// ===========================================================================
// Unblocked Householder on panel [col0, col0+w) of A, rows col0..m-1, one
// workgroup of 512 threads per item.  Each column costs one pass over the
// remaining panel rows: the pass applies reflector j to columns j+1.. and, on
// the fly, accumulates the squared norm of the next column below its diagonal
// and the unscaled products of that column with the later ones; one block
// reduction then gives every scalar the next reflector needs.
constexpr int PANEL_THREADS = 512;

__device__ __forceinline__ void panel_reduce(double (&part)[QR_NB + 1], int nval, double (*red)[QR_NB + 2],
                                             double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c <= QR_NB; ++c) {
        if (c < nval) {
            const double v = wave_sum(part[c]);
            if (lane == 0) red[wv][c] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nval) {
        double sum = 0.0;
        for (int q = 0; q < PANEL_THREADS / 64; ++q) sum += red[q][threadIdx.x];
        out[threadIdx.x] = sum;
    }
    __syncthreads();
}

// Columns [jb, je) of the panel, one pass each, updating columns < wl.  On
// entry sh[0] is the squared norm of column jb below its diagonal and
// sh[1 + k] its product with column jb + 1 + k (rows below the diagonal).
__device__ __forceinline__ void panel_cols(const QRItem& it, int col0, double* V, int64_t ld, int mp, int jb,
                                           int je, int wl, double (*red)[QR_NB + 2], double* sh, double* coef) {
    double part[QR_NB + 1];
    for (int j = jb; j < je; ++j) {
        // reflector j from alpha = V[j][j] and ||x[1:]||^2 = sh[0], formed by
        // every thread alike; thread c - j - 1 forms the coefficient of column c
        const double alpha = V[j + j * ld];
        const double xn2 = sh[0];
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        {
            // coefficient tau * (v . a_c), v = [1; scal * x[1:]]
            const int c = j + 1 + (int)threadIdx.x;
            if (c < wl) coef[c] = tau * (V[j + c * ld] + scal * sh[1 + threadIdx.x]);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            it.tau[col0 + j] = tau;
            V[j + j * ld] = beta;
        }
#pragma unroll
        for (int c = 0; c <= QR_NB; ++c) part[c] = 0.0;
        // one pass: scale v, update columns j+1..wl-1, accumulate for column
        // j+1.  All of a row's loads are issued before its first store, so
        // they are in flight together.
        for (int r = j + threadIdx.x; r < mp; r += PANEL_THREADS) {
            double x[QR_NB];
            const double* row = V + r + (int64_t)j * ld;
#pragma unroll
            for (int c = 0; c < QR_NB; ++c) x[c] = (j + c < wl) ? row[(int64_t)c * ld] : 0.0;
            double v = 1.0;
            if (r > j) {
                v = x[0] * scal;
                V[r + j * ld] = v;
            }
            double xn = 0.0;
#pragma unroll
            for (int c = 1; c < QR_NB; ++c) {
                const int cc = j + c;
                if (cc < wl) {
                    const double a = x[c] - coef[cc] * v;
                    V[r + cc * ld] = a;
                    if (c == 1) {
                        xn = a;
                        if (r > j + 1) part[0] += a * a;
                    } else if (r > j + 1) {
                        part[c - 1] += xn * a;
                    }
                }
            }
        }
        __syncthreads();
        if (j + 1 < je) panel_reduce(part, wl - j - 1, red, sh);
    }
}

// The panel is factored in two halves of QR_HB columns: the first half by
// the column passes above (touching only its own columns), then one pass
// applies its reflectors to the second half in compact WY form,
// A2 -= V1 T1^T (V1^T A2) (G1 = V1^T V1 and V1^T A2 by MFMA), and the second
// half is factored.  Each pass over the panel thus moves about a third fewer
// bytes than column passes over all 32 columns.
constexpr int QR_HB = 16;

__global__ void __launch_bounds__(PANEL_THREADS) k_qr_panel(const QRItem* q, int nitems, int col0) {
    __shared__ double red[PANEL_THREADS / 64][QR_NB + 2];
    __shared__ double sh[QR_NB + 2];  // sh[0] = norm^2 below diag of the current column, sh[1+k] = dots
    __shared__ double coef[QR_NB];
    __shared__ double gz[2][PANEL_THREADS / 64][QR_HB * QR_HB];
    __shared__ double G1[QR_HB][QR_HB + 1], Z1[QR_HB][QR_HB + 1], T1[QR_HB][QR_HB + 1], M1[QR_HB][QR_HB + 1];
    const int b = blockIdx.x;
    if (b >= nitems) return;
    const QRItem it = q[b];
    if (it.nfac <= col0 || it.A.m <= col0) return;
    const int w = min(QR_NB, it.nfac - col0);
    const int mp = qr_rows(it.A.m, it.zrow, it.zslope, col0, QR_NB) - col0;
    const int64_t ld = it.A.ld;
    double* V = it.A.p + col0 + (int64_t)col0 * ld;
    const int w1 = (w > QR_HB) ? QR_HB : w;  // first half
    double part[QR_NB + 1];
    // column 0: norm^2 of x[1:] and products x[1:] . a_c[1:], c = 1..w1-1
#pragma unroll
    for (int c = 0; c <= QR_NB; ++c) part[c] = 0.0;
    for (int r = 1 + threadIdx.x; r < mp; r += PANEL_THREADS) {
        const double x = V[r];
        part[0] += x * x;
#pragma unroll
        for (int c = 1; c < QR_HB; ++c)
            if (c < w1) part[c] += x * V[r + c * ld];
    }
    panel_reduce(part, w1, red, sh);
    panel_cols(it, col0, V, ld, mp, 0, w1, w1, red, sh, coef);
    if (w <= QR_HB) return;

    // second half: G1 = V1^T V1, Z1 = V1^T A2 (V1 unit lower trapezoid)
    const int w2 = w - QR_HB;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    {
        double4_t ag = {0.0, 0.0, 0.0, 0.0}, az = {0.0, 0.0, 0.0, 0.0};
        const int k = lane & 15;
#pragma unroll 4
        for (int r0 = 4 * wv; r0 < mp; r0 += 4 * (PANEL_THREADS / 64)) {
            const int r = r0 + (lane >> 4);
            double v = 0.0, a2 = 0.0;
            if (r < mp) {
                v = (r < k) ? 0.0 : (r == k ? 1.0 : V[r + k * ld]);
                if (k < w2) a2 = V[r + (QR_HB + k) * ld];
            }
            ag = mfma_f64(v, v, ag);
            az = mfma_f64(v, a2, az);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ij = (4 * e + (lane >> 4)) * QR_HB + (lane & 15);
            gz[0][wv][ij] = ag[e];
            gz[1][wv][ij] = az[e];
        }
    }
    __syncthreads();
    if (threadIdx.x < QR_HB * QR_HB) {
        const int e = threadIdx.x;
        double g = 0.0, z = 0.0;
        for (int q2 = 0; q2 < PANEL_THREADS / 64; ++q2) {
            g += gz[0][q2][e];
            z += gz[1][q2][e];
        }
        G1[e / QR_HB][e % QR_HB] = g;
        Z1[e / QR_HB][e % QR_HB] = z;
        T1[e / QR_HB][e % QR_HB] = 0.0;
    }
    __syncthreads();
    // T1(0:j, j) = -tau_j T1(0:j, 0:j) G1(0:j, j), T1(j, j) = tau_j
    for (int j = 0; j < QR_HB; ++j) {
        const double tj = it.tau[col0 + j];
        if ((int)threadIdx.x < j) {
            const int i = threadIdx.x;
            double sum = 0.0;
            for (int l = i; l < j; ++l) sum += T1[i][l] * G1[l][j];
            T1[i][j] = -tj * sum;
        }
        if (threadIdx.x == 0) T1[j][j] = tj;
        __syncthreads();
    }
    // M1 = T1^T Z1
    if (threadIdx.x < QR_HB * QR_HB) {
        const int kk = threadIdx.x / QR_HB, c = threadIdx.x % QR_HB;
        double sum = 0.0;
        for (int i = 0; i <= kk; ++i) sum += T1[i][kk] * Z1[i][c];
        M1[kk][c] = sum;
    }
    __syncthreads();
    // A2 -= V1 M1 on MFMA (a wave takes 16-row blocks; lane l ends with
    // A2(r0 + 4e + l/16, l%16)), and the sums that start the second half:
    // each lane accumulates column QR_HB times its own column
    {
        const int li = lane & 15, lq = lane >> 4;
        double bm[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) bm[s4] = M1[4 * s4 + lq][li];
        double pc = 0.0;
        for (int r0 = 16 * wv; r0 < mp; r0 += 16 * (PANEL_THREADS / 64)) {
            double4_t acc = {0.0, 0.0, 0.0, 0.0};
            double a2[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = r0 + 4 * e + lq;
                a2[e] = (r < mp && li < w2) ? V[r + (int64_t)(QR_HB + li) * ld] : 0.0;
            }
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int r = r0 + li, k = 4 * s4 + lq;
                double v = 0.0;
                if (r < mp) v = (r < k) ? 0.0 : (r == k ? 1.0 : V[r + (int64_t)k * ld]);
                acc = mfma_f64(v, bm[s4], acc);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = r0 + 4 * e + lq;
                double a = 0.0;
                if (r < mp && li < w2) {
                    a = a2[e] - acc[e];
                    V[r + (int64_t)(QR_HB + li) * ld] = a;
                }
                const double a0 = __shfl(a, lane & 0x30, 64);  // column QR_HB of the same row
                if (r > QR_HB) pc += a0 * a;
            }
        }
#pragma unroll
        for (int c = 0; c <= QR_NB; ++c) part[c] = (c == li) ? pc : 0.0;
    }
    __syncthreads();
    panel_reduce(part, w2, red, sh);
    panel_cols(it, col0, V, ld, mp, QR_HB, w, w, red, sh, coef);
}

// T factor for the reflectors of panel k: T = upper triangular with
// H_0 ... H_{w-1} = I - V T V^T, from G = V^T V over rows col0..m-1.  G is
// summed from partials over chunks of QR_GKS rows (MFMA, many workgroups per
// item), then one workgroup per item runs the recurrence
// T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j), T(j, j) = tau_j.
constexpr int QR_GKS = 256;

struct OpPanelGram {
    const ORItem* o;
    double* const* Wp;  // per item: ceil(mp / QR_GKS) partials of 32 x 32
    int col0;
    __device__ int mrows(int b) const { return qr_rows(o[b].V.m, o[b].zrow, o[b].zslope, col0, QR_NB) - col0; }
    __device__ int tiles(int b) const {
        if (o[b].V.n <= col0 || o[b].V.m <= col0) return 0;
        return (mrows(b) + QR_GKS - 1) / QR_GKS;
    }
    __device__ void operator()(int b, int ks) const {
        __shared__ double Vs[4][64][QR_NB + 1];
        const ORItem& it = o[b];
        const int w = min(QR_NB, it.V.n - col0);
        const int mp = mrows(b);
        const int64_t ld = it.V.ld;
        const double* V = it.V.p + col0 + (int64_t)col0 * ld;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        // wave wv stages rows ks*QR_GKS + 64 wv + lane (unit lower trapezoid)
        const int gr = ks * QR_GKS + wv * 64 + lane;
#pragma unroll 8
        for (int c = 0; c < QR_NB; ++c) {
            double v = 0.0;
            if (gr < mp && c < w) v = (gr < c) ? 0.0 : (gr == c ? 1.0 : V[gr + (int64_t)c * ld]);
            Vs[wv][lane][c] = v;
        }
        __syncthreads();
        double4_t acc[2][2];
        acc_zero(acc);
#pragma unroll 4
        for (int kq = 0; kq < 16; ++kq) {
            const int kk = kq * 4 + (lane >> 4);
            const double a0 = Vs[wv][kk][lane & 15], a1 = Vs[wv][kk][16 + (lane & 15)];
            acc[0][0] = mfma_f64(a0, a0, acc[0][0]);
            acc[0][1] = mfma_f64(a0, a1, acc[0][1]);
            acc[1][0] = mfma_f64(a1, a0, acc[1][0]);
            acc[1][1] = mfma_f64(a1, a1, acc[1][1]);
        }
        __syncthreads();
        double* red = &Vs[0][0][0];  // 4 x 1024 doubles
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    red[wv * 1024 + (16 * x + 4 * e + (lane >> 4)) + 32 * (16 * y + (lane & 15))] = acc[x][y][e];
        __syncthreads();
        double* P = Wp[b] + (int64_t)ks * 1024;
        for (int e = threadIdx.x; e < 1024; e += 256) P[e] = (red[e] + red[1024 + e]) + (red[2048 + e] + red[3072 + e]);
    }
};

struct OpBuildT {
    const ORItem* o;
    const double* const* tau;  // per item tau array (reflector j's tau at tau[b][j])
    double* const* Wp;         // Gram partials from OpPanelGram
    int col0;
    __device__ int tiles(int b) const { return (o[b].V.n > col0 && o[b].V.m > col0) ? 1 : 0; }
    __device__ void operator()(int b, int) const {
        __shared__ double G[32][33];
        __shared__ double T[32][33];
        const DMat Vm = o[b].V;
        const int w = min(QR_NB, Vm.n - col0);
        const int mp = qr_rows(Vm.m, o[b].zrow, o[b].zslope, col0, QR_NB) - col0;
        const int nks = (mp + QR_GKS - 1) / QR_GKS;
        const double* P = Wp[b];
        for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
            double sum = 0.0;
            for (int ks = 0; ks < nks; ++ks) sum += P[(int64_t)ks * 1024 + e];
            G[e & 31][e >> 5] = sum;
        }
        for (int e = threadIdx.x; e < 32 * 33; e += blockDim.x) (&T[0][0])[e] = 0.0;
        __syncthreads();
        const double* tb = tau[b] + col0;
        for (int j = 0; j < w; ++j) {
            const double tj = tb[j];
            if (threadIdx.x < j) {
                const int i = threadIdx.x;
                double sum = 0.0;
                for (int l = i; l < j; ++l) sum += T[i][l] * G[l][j];
                T[i][j] = -tj * sum;
            }
            if (threadIdx.x == 0) T[j][j] = tj;
            __syncthreads();
        }
        double* To = o[b].T + (int64_t)(col0 / QR_NB) * QR_NB * QR_NB;
        for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
            const int r = e & 31, c = e >> 5;
            To[r + c * 32] = T[r][c];
        }
    }
};

// ---------------------------------------------------------------------------
// Block application of reflectors.  A block is up to four consecutive
// 32-column panels starting at column c0 of V (width wb <= 128).  For C over
// a column range [cc0, cc1):
//   P = V_b^T C                     (row chunks of QR_KS rows -> partial sums)
//   W = recurrence over the panels  (TRANS: W_q = T_q^T (P_q - sum_{j<q} G_qj W_j),
//                                    else:  W_q = T_q (P_q - sum_{j>q} G_qj W_j))
//   C -= V_b W
// which applies H_0^T..H_3^T (TRANS) or H_3..H_0 in turn while reading C twice.
// ---------------------------------------------------------------------------
constexpr int QR_KS = 2048;

struct BlkRange {  // per-item column range and width of the current block
    int wb, cc0, cc1;
};
// mode 0: ormqr (all columns); mode 1: geqrf trailing [c0+wb, n); mode 2: geqrf
// inner [c0+wb, min(n, oend, nfac)) (the factored columns of the current outer block)
__device__ __forceinline__ BlkRange blk_range(const ORItem& it, int c0, int cap, int mode, int oend) {
    BlkRange r;
    r.wb = min(cap, it.V.n - c0);
    if (mode == 0) { r.cc0 = 0; r.cc1 = it.C.n; }
    else if (mode == 1) { r.cc0 = c0 + r.wb; r.cc1 = it.C.n; }
    else if (mode == 2) { r.cc0 = c0 + r.wb; r.cc1 = min(min(it.C.n, oend), it.V.n); }  // inner: factored columns only
    else { r.cc0 = c0; r.cc1 = it.C.n; }  // explicit Q: columns left of the block are still unit vectors
    return r;
}

// P partial sums (nks slabs) and W use leading dimension QR_PAIR: a 256-column
// pair of reflector blocks is applied to C in one pass (see apply_pair).
constexpr int PLD = QR_PAIR;

struct BlkOp {
    const ORItem* o;
    double* const* Wp;  // per item partial sums: nks x PLD x max(PLD, C.n)
    int c0, cap, mode, oend;
    int half = 0;       // OpBlkW / OpBlkCorr: which 128-block of a pair
    __device__ bool active(int b, BlkRange& r) const {
        if (o[b].V.n <= c0 || o[b].V.m <= c0) return false;
        r = blk_range(o[b], c0, cap, mode, oend);
        return r.wb > 0 && r.cc1 > r.cc0;
    }
    __device__ int mrows(int b) const { return qr_rows(o[b].V.m, o[b].zrow, o[b].zslope, c0, cap) - c0; }
    __device__ int nks(int b) const { return (mrows(b) + QR_KS - 1) / QR_KS; }
    __device__ int pstride(int b) const { return PLD * max(PLD, o[b].C.n); }
};

// P partials: tile = (row tile of the block 64, column tile 64, row chunk)
struct OpBlkP : BlkOp {
    __device__ int tiles(int b) const {
        BlkRange r;
        if (!active(b, r)) return 0;
        return ((r.wb + 63) / 64) * ((r.cc1 - r.cc0 + 63) / 64) * nks(b);
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmem sm;
        BlkRange R;
        active(b, R);
        const ORItem& it = o[b];
        const int nc = R.cc1 - R.cc0;
        const int ntc = (nc + 63) / 64, ntr = (R.wb + 63) / 64;
        const int tr = t % ntr, tc = (t / ntr) % ntc, ks = t / (ntr * ntc);
        const int mp = mrows(b);
        const int r0 = ks * QR_KS;
        const int kl = min(QR_KS, mp - r0);
        const double* V = it.V.p + c0 + r0 + (int64_t)c0 * it.V.ld;
        const double* C = it.C.p + c0 + r0 + (int64_t)R.cc0 * it.C.ld;
        double4_t acc[2][2];
        acc_zero(acc);
        if (ks == 0) mfma_tile_64<true, false, 1, 0>(V, it.V.ld, C, it.C.ld, R.wb, nc, kl, tr * 64, tc * 64, sm, acc);
        else mfma_tile_64<true, false, 0, 0>(V, it.V.ld, C, it.C.ld, R.wb, nc, kl, tr * 64, tc * 64, sm, acc);
        double* P = Wp[b] + (int64_t)ks * pstride(b);
        acc_foreach(acc, [&](int r, int c, double v) {
            const int gr = tr * 64 + r, gc = tc * 64 + c;
            if (gr < R.wb && gc < nc) P[gr + (int64_t)gc * PLD] = v;
        });
    }
};

// the row tiles of one column tile and row chunk are consecutive tiles and
// read the same block of C: XCD-chunked mappings keep them in one L2
template <>
struct XcdChunked<OpBlkP> {
    static constexpr bool value = true;
};

// W from the summed partials for one 128-block (half of the range), per
// 64-column tile: W_q = T_q^T (P_q - sum_j G_qj W_j) over its 32-column panels
// (T_q (P_q - ...) for Q C)
template <bool TRANS>
struct OpBlkW : BlkOp {
    __device__ int tiles(int b) const {
        BlkRange r;
        if (!active(b, r)) return 0;
        if (r.wb - QR_OB * half <= 0) return 0;
        return (r.cc1 - r.cc0 + 63) / 64;
    }
    __device__ void operator()(int b, int t) const {
        __shared__ double P[QR_OB][65];
        BlkRange R;
        active(b, R);
        const ORItem& it = o[b];
        const int nc = R.cc1 - R.cc0;
        const int j0 = t * 64;
        const int nks_ = nks(b);
        const int ps = pstride(b);
        const int roff = QR_OB * half, c0h = c0 + roff;
        const int wbh = min(QR_OB, R.wb - roff);
        const int nsub = (wbh + QR_NB - 1) / QR_NB;
        for (int e = threadIdx.x; e < QR_OB * 64; e += blockDim.x) {
            const int r = e & (QR_OB - 1), c = e >> 7;
            double sum = 0.0;
            if (r < wbh && j0 + c < nc)
                for (int ks = 0; ks < nks_; ++ks) sum += Wp[b][(int64_t)ks * ps + (roff + r) + (int64_t)(j0 + c) * PLD];
            P[r][c] = sum;
        }
        __syncthreads();
        // MFMA 16x16x4: wave wv owns rows 16 (wv & 1) .. +15 of the current
        // panel and the column blocks 2 (wv >> 1), 2 (wv >> 1) + 1 of the tile
        const double* Tg0 = it.T + (int64_t)(c0h / QR_NB) * QR_NB * QR_NB;
        const double* Gg = it.G + (int64_t)(c0h / QR_OB) * QR_OB * QR_OB;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int rb = wv & 1, cb0 = (wv >> 1) * 2;
        const int li = lane & 15, lk = lane >> 4;
        for (int step = 0; step < nsub; ++step) {
            const int q = TRANS ? step : nsub - 1 - step;
            const int wq = min(QR_NB, wbh - 32 * q);
            double4_t acc[2];
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[y][e] = P[32 * q + 16 * rb + 4 * e + lk][16 * (cb0 + y) + li];
            // U_q = P_q - sum over the panels already turned into W of G_qj W_j
            // (the lower blocks of the Gram: G(32q + i, 32j + k) for j < q, or
            // G(32j + k, 32q + i) for j > q)
            const int jb = TRANS ? 0 : q + 1, je = TRANS ? q : nsub;
            for (int j = jb; j < je; ++j) {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    const int gi = 32 * q + 16 * rb + li, gk = 32 * j + 4 * kk + lk;
                    double a = 0.0;
                    if (gi < wbh && gk < wbh) a = -(TRANS ? Gg[gi + (int64_t)gk * QR_OB] : Gg[gk + (int64_t)gi * QR_OB]);
#pragma unroll
                    for (int y = 0; y < 2; ++y) acc[y] = mfma_f64(a, P[gk][16 * (cb0 + y) + li], acc[y]);
                }
            }
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 16 * rb + 4 * e + lk;
                    P[32 * q + r][16 * (cb0 + y) + li] = (r < wq) ? acc[y][e] : 0.0;
                }
            __syncthreads();
            // W_q = T_q^T U_q (T_q U_q for Q C); T_q is zero outside its wq x wq corner
            double4_t acc2[2] = {double4_t{0.0, 0.0, 0.0, 0.0}, double4_t{0.0, 0.0, 0.0, 0.0}};
            const double* Tq = Tg0 + (int64_t)q * QR_NB * QR_NB;
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int i_ = 16 * rb + li, k_ = 4 * kk + lk;
                const double a = TRANS ? Tq[k_ + 32 * i_] : Tq[i_ + 32 * k_];
#pragma unroll
                for (int y = 0; y < 2; ++y) acc2[y] = mfma_f64(a, P[32 * q + k_][16 * (cb0 + y) + li], acc2[y]);
            }
            __syncthreads();
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int e = 0; e < 4; ++e) P[32 * q + 16 * rb + 4 * e + lk][16 * (cb0 + y) + li] = acc2[y][e];
            __syncthreads();
        }
        for (int e = threadIdx.x; e < QR_OB * 64; e += blockDim.x) {
            const int r = e & (QR_OB - 1), c = e >> 7;
            if (r < wbh && j0 + c < nc) it.W[(roff + r) + (int64_t)(j0 + c) * PLD] = P[r][c];
        }
    }
};

// Coupling of the two blocks of a pair before the second W: with the cross
// Gram Gx = V_b^T V_a, C <- Q^T C needs P_b -= Gx W_a (W_a first), and
// C <- Q C needs P_a -= Gx^T W_b (W_b first).  Applied to partial slab 0.
template <bool TRANS>
struct OpBlkCorr : BlkOp {
    __device__ int tiles(int b) const {
        BlkRange r;
        if (!active(b, r) || r.wb <= QR_OB) return 0;
        const int wt = TRANS ? r.wb - QR_OB : QR_OB;
        return ((wt + 63) / 64) * ((r.cc1 - r.cc0 + 63) / 64);
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmem sm;
        BlkRange R;
        active(b, R);
        const ORItem& it = o[b];
        const int nc = R.cc1 - R.cc0;
        const int wa = QR_OB, wbb = R.wb - QR_OB;
        const int wt = TRANS ? wbb : wa, ws = TRANS ? wa : wbb;    // target / source widths
        const int rt = TRANS ? QR_OB : 0, rs = TRANS ? 0 : QR_OB;  // their row offsets in P and W
        const int tm = (wt + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        const int nblk = (it.V.n + QR_OB - 1) / QR_OB;
        const double* Gx = it.G + (int64_t)(nblk + c0 / QR_PAIR) * QR_OB * QR_OB;
        double4_t acc[2][2];
        acc_zero(acc);
        mfma_tile_64<!TRANS, false>(Gx, QR_OB, it.W + rs, PLD, wt, nc, ws, i0, j0, sm, acc);
        double* P0 = Wp[b];
        acc_foreach(acc, [&](int r, int c, double v) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < wt && gj < nc) P0[(rt + gi) + (int64_t)gj * PLD] -= v;
        });
    }
};

// C -= V_b W
struct OpBlkUpd : BlkOp {
    __device__ int tiles(int b) const {
        BlkRange r;
        if (!active(b, r)) return 0;
        const int mp = mrows(b);
        return ((mp + 63) / 64) * ((r.cc1 - r.cc0 + 63) / 64);
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemC sm;
        BlkRange R;
        active(b, R);
        const ORItem& it = o[b];
        const int mp = mrows(b);
        const int nc = R.cc1 - R.cc0;
        // 8 x 8 groups of tiles: bands of 8 row tiles, each band swept in
        // groups of 8 column tiles (column fastest), so that 64 consecutive
        // tiles read 8 panels of V_b and 8 panels of W
        const int tm = (mp + 63) / 64, tn = (nc + 63) / 64;
        const int band = t / (8 * tn), r = t - band * 8 * tn;
        const int rows = min(8, tm - band * 8);
        const int cg = r / (rows * 8), q = r - cg * rows * 8;
        const int cols = min(8, tn - cg * 8);
        const int i0 = (band * 8 + q / cols) * 64, j0 = (cg * 8 + q % cols) * 64;
        const double* V = it.V.p + c0 + (int64_t)c0 * it.V.ld;
        double* C = it.C.p + c0 + (int64_t)R.cc0 * it.C.ld;
        const int ld = it.C.ld;
        double4_t acc[2][2];
        acc_zero(acc);
        // row tiles below the block's unit trapezoid read V_b as a plain operand
        if (i0 >= R.wb) mfma_tile_64<false, false, 0, 0>(V, it.V.ld, it.W, PLD, mp, nc, R.wb, i0, j0, sm.t, acc);
        else mfma_tile_64<false, false, 1, 0>(V, it.V.ld, it.W, PLD, mp, nc, R.wb, i0, j0, sm.t, acc);
        acc_store_coalesced(acc, sm, [&](int r, int c, double v) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < mp && gj < nc) C[gi + (int64_t)gj * ld] -= v;
        });
    }
};

template <>
struct XcdChunked<OpBlkUpd> {
    static constexpr bool value = true;
};

// G = V_b^T V_b for the 128-column block at c0 (partials then ordered sum)
struct OpGramP : BlkOp {
    __device__ int tiles(int b) const {
        if (o[b].V.n <= c0 || o[b].V.m <= c0) return 0;
        const int wb = min(QR_OB, o[b].V.n - c0);
        if (wb <= QR_NB) return 0;
        const int T = (wb + 63) / 64;
        return T * T * nks(b);
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmem sm;
        const ORItem& it = o[b];
        const int wb = min(QR_OB, it.V.n - c0);
        const int T = (wb + 63) / 64;
        const int tr = t % T, tc = (t / T) % T, ks = t / (T * T);
        const int mp = mrows(b);
        const int r0 = ks * QR_KS;
        const int kl = min(QR_KS, mp - r0);
        const double* V = it.V.p + c0 + r0 + (int64_t)c0 * it.V.ld;
        double4_t acc[2][2];
        acc_zero(acc);
        if (ks == 0) mfma_tile_64<true, false, 1, 1>(V, it.V.ld, V, it.V.ld, wb, wb, kl, tr * 64, tc * 64, sm, acc);
        else mfma_tile_64<true, false, 0, 0>(V, it.V.ld, V, it.V.ld, wb, wb, kl, tr * 64, tc * 64, sm, acc);
        double* P = Wp[b] + (int64_t)ks * pstride(b);
        acc_foreach(acc, [&](int r, int c, double v) {
            const int gr = tr * 64 + r, gc = tc * 64 + c;
            if (gr < wb && gc < wb) P[gr + (int64_t)gc * QR_OB] = v;
        });
    }
};
struct OpGramR : BlkOp {
    __device__ int tiles(int b) const {
        return (o[b].V.n > c0 && o[b].V.m > c0 && min(QR_OB, o[b].V.n - c0) > QR_NB) ? 1 : 0;
    }
    __device__ void operator()(int b, int) const {
        const ORItem& it = o[b];
        const int wb = min(QR_OB, it.V.n - c0);
        const int nks_ = nks(b);
        const int ps = pstride(b);
        double* G = it.G + (int64_t)(c0 / QR_OB) * QR_OB * QR_OB;
        for (int e = threadIdx.x; e < QR_OB * QR_OB; e += blockDim.x) {
            const int r = e & (QR_OB - 1), c = e >> 7;
            double sum = 0.0;
            if (r < wb && c < wb)
                for (int ks = 0; ks < nks_; ++ks) sum += Wp[b][(int64_t)ks * ps + r + (int64_t)c * QR_OB];
            G[r + (int64_t)c * QR_OB] = sum;
        }
    }
};

struct QrScratch {
    DBuf<double> buf;
    DBuf<double*> ptr;
    void alloc(const std::vector<ORItem>& items, hipStream_t s) {
        std::vector<int64_t> off(items.size() + 1, 0);
        for (size_t i = 0; i < items.size(); ++i) {
            const int nks = ceil_div(std::max(1, items[i].V.m), QR_KS);
            off[i + 1] = off[i] + (int64_t)PLD * std::max(PLD, items[i].C.n) * nks;
        }
        buf.alloc(off.back());
        std::vector<double*> hp(items.size());
        for (size_t i = 0; i < items.size(); ++i) hp[i] = buf.p + off[i];
        ptr.alloc(hp.size());
        h2d(ptr.p, hp.data(), hp.size(), s);
        DD_HIP(hipStreamSynchronize(s));
    }
};

// T factor of the 32-column panel at col0 (Gram partials in the scratch)
static void build_t_panel(Batch<ORItem>& o, QrScratch& sc, const double* const* dtau, int col0, hipStream_t s) {
    int64_t ng = 0, nt = 0;
    for (auto& x : o.h) {
        if (x.V.n <= col0 || x.V.m <= col0) continue;
        ++nt;
        ng += ceil_div(qr_rows(x.V.m, x.zrow, x.zslope, col0, QR_NB) - col0, QR_GKS);
    }
    if (nt == 0) return;
    launch_tiles(OpPanelGram{o.d.p, sc.ptr.p, col0}, o.size(), ng, s, "qr_panel_gram");
    launch_tiles(OpBuildT{o.d.p, dtau, sc.ptr.p, col0}, o.size(), nt, s, "qr_buildT");
}

static void apply_block(Batch<ORItem>& o, QrScratch& sc, int c0, int cap, int mode, int oend, bool trans,
                        hipStream_t s) {
    int64_t np = 0, nw = 0, nu = 0;
    for (auto& x : o.h) {
        if (x.V.n <= c0 || x.V.m <= c0) continue;
        const int wb = std::min(cap, x.V.n - c0);
        int cc0, cc1;
        if (mode == 0) { cc0 = 0; cc1 = x.C.n; }
        else if (mode == 1) { cc0 = c0 + wb; cc1 = x.C.n; }
        else if (mode == 2) { cc0 = c0 + wb; cc1 = std::min(std::min(x.C.n, oend), x.V.n); }
        else { cc0 = c0; cc1 = x.C.n; }
        if (wb <= 0 || cc1 <= cc0) continue;
        const int ntc = ceil_div(cc1 - cc0, 64);
        const int mp = qr_rows(x.V.m, x.zrow, x.zslope, c0, cap) - c0;
        nw += ntc;
        np += (int64_t)ceil_div(wb, 64) * ntc * ceil_div(mp, QR_KS);
        nu += (int64_t)ceil_div(mp, 64) * ntc;
    }
    if (nw == 0) return;
    BlkOp base{o.d.p, sc.ptr.p, c0, cap, mode, oend};
    launch_tiles(OpBlkP{base}, o.size(), np, s, "qr_blk_p");
    if (trans) launch_tiles(OpBlkW<true>{base}, o.size(), nw, s, "qr_blk_w");
    else launch_tiles(OpBlkW<false>{base}, o.size(), nw, s, "qr_blk_w");
    // Algorithmic work of C -= V_b W: V_b is a unit lower trapezoid with
    // mp*wb - wb(wb-1)/2 structural entries, so 2*nc flops per entry; bytes =
    // read the strictly lower part of V_b and W once, read and write C once.
    auto work = [&](int b0, int cnt, double& fl, double& by) {
        for (int i = b0; i < b0 + cnt; ++i) {
            const ORItem& x = o.h[i];
            if (x.V.n <= c0 || x.V.m <= c0) continue;
            const int wb = std::min(cap, x.V.n - c0);
            int cc0, cc1;
            if (mode == 0) { cc0 = 0; cc1 = x.C.n; }
            else if (mode == 1) { cc0 = c0 + wb; cc1 = x.C.n; }
            else if (mode == 2) { cc0 = c0 + wb; cc1 = std::min(std::min(x.C.n, oend), x.V.n); }
            else { cc0 = c0; cc1 = x.C.n; }
            if (wb <= 0 || cc1 <= cc0) continue;
            const double mp = qr_rows(x.V.m, x.zrow, x.zslope, c0, cap) - c0, nc = cc1 - cc0;
            const double nzv = mp * wb - 0.5 * wb * (wb - 1.0);
            fl += 2.0 * nc * nzv;
            by += 8.0 * ((nzv - wb) + (double)wb * nc + 2.0 * mp * nc);
        }
    };
    launch_tiles(OpBlkUpd{base}, o.size(), nu, s, "qr_blk_upd", 4096, work);
}

static void gram_block(Batch<ORItem>& o, QrScratch& sc, int c0, hipStream_t s) {
    int64_t np = 0, nr = 0;
    for (auto& x : o.h) {
        if (x.V.n <= c0 || x.V.m <= c0) continue;
        const int wb = std::min(QR_OB, x.V.n - c0);
        if (wb <= QR_NB) continue;  // a single panel needs no G
        const int T = ceil_div(wb, 64);
        np += (int64_t)T * T * ceil_div(qr_rows(x.V.m, x.zrow, x.zslope, c0, QR_OB) - c0, QR_KS);
        ++nr;
    }
    if (nr == 0) return;
    BlkOp base{o.d.p, sc.ptr.p, c0, QR_OB, 0, 0};
    launch_tiles(OpGramP{base}, o.size(), np, s, "qr_gram_p");
    launch_tiles(OpGramR{base}, o.size(), nr, s, "qr_gram_r");
}

// Cross Gram Gx = V_b^T V_a of the pair (a at c0, b at c0 + 128): both vanish
// above row c0 + 128 except V_a, whose rows there are all below its diagonal.
// Partials over row chunks, then an ordered sum (rows of Gx past V_b's width are 0).
struct OpGramXP : BlkOp {
    __device__ int wbb(int b) const { return min(QR_OB, o[b].V.n - c0 - QR_OB); }
    __device__ int mx(int b) const { return qr_rows(o[b].V.m, o[b].zrow, o[b].zslope, c0 + QR_OB, QR_OB) - (c0 + QR_OB); }
    __device__ int tiles(int b) const {
        if (o[b].V.n <= c0 + QR_OB || mx(b) <= 0) return 0;
        return ((wbb(b) + 63) / 64) * 2 * ((mx(b) + QR_KS - 1) / QR_KS);
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmem sm;
        const ORItem& it = o[b];
        const int wb = wbb(b), m = mx(b);
        const int tr = t % ((wb + 63) / 64), rest = t / ((wb + 63) / 64);
        const int tc = rest % 2, ks = rest / 2;
        const int r0 = ks * QR_KS, kl = min(QR_KS, m - r0);
        const int cb = c0 + QR_OB;
        const double* Vb = it.V.p + cb + r0 + (int64_t)cb * it.V.ld;
        const double* Va = it.V.p + cb + r0 + (int64_t)c0 * it.V.ld;
        double4_t acc[2][2];
        acc_zero(acc);
        if (ks == 0) mfma_tile_64<true, false, 1, 0>(Vb, it.V.ld, Va, it.V.ld, wb, QR_OB, kl, tr * 64, tc * 64, sm, acc);
        else mfma_tile_64<true, false, 0, 0>(Vb, it.V.ld, Va, it.V.ld, wb, QR_OB, kl, tr * 64, tc * 64, sm, acc);
        double* P = Wp[b] + (int64_t)ks * pstride(b);
        acc_foreach(acc, [&](int r, int c, double v) {
            const int gr = tr * 64 + r, gc = tc * 64 + c;
            if (gr < wb && gc < QR_OB) P[gr + (int64_t)gc * QR_OB] = v;
        });
    }
};
struct OpGramXR : BlkOp {
    __device__ int tiles(int b) const { return o[b].V.n > c0 + QR_OB ? 1 : 0; }
    __device__ void operator()(int b, int) const {
        const ORItem& it = o[b];
        const int wb = min(QR_OB, it.V.n - c0 - QR_OB);
        const int m = qr_rows(it.V.m, it.zrow, it.zslope, c0 + QR_OB, QR_OB) - (c0 + QR_OB);
        const int nks_ = m > 0 ? (m + QR_KS - 1) / QR_KS : 0;
        const int ps = pstride(b);
        const int nblk = (it.V.n + QR_OB - 1) / QR_OB;
        double* Gx = it.G + (int64_t)(nblk + c0 / QR_PAIR) * QR_OB * QR_OB;
        for (int e = threadIdx.x; e < QR_OB * QR_OB; e += blockDim.x) {
            const int r = e & (QR_OB - 1), c = e >> 7;
            double sum = 0.0;
            if (r < wb)
                for (int ks = 0; ks < nks_; ++ks) sum += Wp[b][(int64_t)ks * ps + r + (int64_t)c * QR_OB];
            Gx[r + (int64_t)c * QR_OB] = sum;
        }
    }
};

static void gram_cross(Batch<ORItem>& o, QrScratch& sc, int c0, hipStream_t s) {
    int64_t np = 0, nr = 0;
    for (auto& x : o.h) {
        if (x.V.n <= c0 + QR_OB) continue;
        const int wbb = std::min(QR_OB, x.V.n - c0 - QR_OB);
        const int m = qr_rows(x.V.m, x.zrow, x.zslope, c0 + QR_OB, QR_OB) - (c0 + QR_OB);
        ++nr;
        if (m > 0) np += (int64_t)ceil_div(wbb, 64) * 2 * ceil_div(m, QR_KS);
    }
    if (nr == 0) return;
    BlkOp base{o.d.p, sc.ptr.p, c0, QR_PAIR, 0, 0};
    if (np) launch_tiles(OpGramXP{base}, o.size(), np, s, "qr_gramx_p");
    launch_tiles(OpGramXR{base}, o.size(), nr, s, "qr_gramx_r");
}

// Q^T C (trans) or Q C for the pair of reflector blocks at c0 and c0 + 128 in
// one pass over C: P = [V_a V_b]^T C, the two W from the 128-block recurrence
// coupled through the cross Gram, then C -= [V_a V_b] [W_a; W_b] with K = 256.
static void apply_pair(Batch<ORItem>& o, QrScratch& sc, int c0, int mode, int oend, bool trans, hipStream_t s) {
    int64_t np = 0, nwa = 0, nwb = 0, ncr = 0, nu = 0;
    for (auto& x : o.h) {
        if (x.V.n <= c0 || x.V.m <= c0) continue;
        const int wb = std::min(QR_PAIR, x.V.n - c0);
        int cc0, cc1;
        if (mode == 0) { cc0 = 0; cc1 = x.C.n; }
        else if (mode == 1) { cc0 = c0 + wb; cc1 = x.C.n; }
        else if (mode == 2) { cc0 = c0 + wb; cc1 = std::min(std::min(x.C.n, oend), x.V.n); }
        else { cc0 = c0; cc1 = x.C.n; }
        if (wb <= 0 || cc1 <= cc0) continue;
        const int ntc = ceil_div(cc1 - cc0, 64);
        const int mp = qr_rows(x.V.m, x.zrow, x.zslope, c0, QR_PAIR) - c0;
        np += (int64_t)ceil_div(wb, 64) * ntc * ceil_div(mp, QR_KS);
        nwa += ntc;
        if (wb > QR_OB) {
            nwb += ntc;
            ncr += (int64_t)ceil_div(trans ? wb - QR_OB : QR_OB, 64) * ntc;
        }
        nu += (int64_t)ceil_div(mp, 64) * ntc;
    }
    if (nwa == 0) return;
    BlkOp base{o.d.p, sc.ptr.p, c0, QR_PAIR, mode, oend};
    BlkOp ha = base, hb = base;
    hb.half = 1;
    launch_tiles(OpBlkP{base}, o.size(), np, s, "qr_blk_p");
    if (trans) {
        launch_tiles(OpBlkW<true>{ha}, o.size(), nwa, s, "qr_blk_w");
        if (ncr) launch_tiles(OpBlkCorr<true>{base}, o.size(), ncr, s, "qr_blk_corr");
        if (nwb) launch_tiles(OpBlkW<true>{hb}, o.size(), nwb, s, "qr_blk_w");
    } else {
        if (nwb) launch_tiles(OpBlkW<false>{hb}, o.size(), nwb, s, "qr_blk_w");
        if (ncr) launch_tiles(OpBlkCorr<false>{base}, o.size(), ncr, s, "qr_blk_corr");
        launch_tiles(OpBlkW<false>{ha}, o.size(), nwa, s, "qr_blk_w");
    }
    auto work = [&](int b0, int cnt, double& fl, double& by) {
        for (int i = b0; i < b0 + cnt; ++i) {
            const ORItem& x = o.h[i];
            if (x.V.n <= c0 || x.V.m <= c0) continue;
            const int wb = std::min(QR_PAIR, x.V.n - c0);
            int cc0, cc1;
            if (mode == 0) { cc0 = 0; cc1 = x.C.n; }
            else if (mode == 1) { cc0 = c0 + wb; cc1 = x.C.n; }
            else if (mode == 2) { cc0 = c0 + wb; cc1 = std::min(std::min(x.C.n, oend), x.V.n); }
            else { cc0 = c0; cc1 = x.C.n; }
            if (wb <= 0 || cc1 <= cc0) continue;
            const double mp = qr_rows(x.V.m, x.zrow, x.zslope, c0, QR_PAIR) - c0, nc = cc1 - cc0;
            const double nzv = mp * wb - 0.5 * wb * (wb - 1.0);
            fl += 2.0 * nc * nzv;
            by += 8.0 * ((nzv - wb) + (double)wb * nc + 2.0 * mp * nc);
        }
    };
    launch_tiles(OpBlkUpd{base}, o.size(), nu, s, "qr_blk_upd", 4096, work);
}

void geqrf_vb(Batch<QRItem>& q, hipStream_t s) {
    int nmax = 0;
    Batch<ORItem> o;
    std::vector<double*> htau;
    for (auto& x : q.h) {
        nmax = std::max(nmax, std::min(x.nfac, x.A.m));
        o.h.push_back(ORItem{DMat{x.A.p, x.A.ld, x.A.m, x.nfac}, x.T, x.A, x.W, x.G, x.zrow, x.zslope});
        htau.push_back(x.tau);
    }
    o.sync(s);
    QrScratch sc;
    sc.alloc(o.h, s);
    DBuf<double*> dtau(htau.size());
    h2d(dtau.p, htau.data(), htau.size(), s);
    for (int col0 = 0; col0 < nmax; col0 += QR_PAIR) {
        for (int sub = 0; sub < 2; ++sub) {
            const int cb = col0 + sub * QR_OB;
            if (cb >= nmax) break;
            for (int in0 = cb; in0 < std::min(nmax, cb + QR_OB); in0 += QR_NB) {
                int64_t np = 0;
                for (auto& x : q.h) np += (x.nfac > in0 && x.A.m > in0) ? 1 : 0;
                if (np) {
                    hipLaunchKernelGGL(k_qr_panel, dim3(q.size()), dim3(PANEL_THREADS), 0, s, q.d.p, q.size(), in0);
                    launch_check("qr_panel");
                }
                build_t_panel(o, sc, dtau.p, in0, s);
                apply_block(o, sc, in0, QR_NB, 2, cb + QR_OB, true, s);  // rest of this 128-block
            }
            gram_block(o, sc, cb, s);
            if (sub == 0) apply_block(o, sc, cb, QR_OB, 2, col0 + QR_PAIR, true, s);  // the pair's second block
        }
        gram_cross(o, sc, col0, s);
        apply_pair(o, sc, col0, 1, 0, true, s);  // trailing matrix
    }
    DD_HIP(hipStreamSynchronize(s));
}

void build_t_vb(Batch<ORItem>& o, const std::vector<double*>& htau, hipStream_t s) {
    int kmax = 0;
    for (auto& x : o.h) kmax = std::max(kmax, x.V.n);
    DBuf<double*> dtau(htau.size());
    h2d(dtau.p, htau.data(), htau.size(), s);
    QrScratch sc;
    sc.alloc(o.h, s);
    for (int col0 = 0; col0 < kmax; col0 += QR_NB) build_t_panel(o, sc, dtau.p, col0, s);
    for (int col0 = 0; col0 < kmax; col0 += QR_OB) gram_block(o, sc, col0, s);
    for (int col0 = 0; col0 < kmax; col0 += QR_PAIR) gram_cross(o, sc, col0, s);
    DD_HIP(hipStreamSynchronize(s));
}

void ormqr_vb(Batch<ORItem>& o, bool trans, hipStream_t s) {
    int kmax = 0;
    for (auto& x : o.h) kmax = std::max(kmax, std::min(x.V.n, x.V.m));
    QrScratch sc;
    sc.alloc(o.h, s);
    const int nb = ceil_div(kmax, QR_PAIR);
    for (int step = 0; step < nb; ++step) {
        const int k = trans ? step : (nb - 1 - step);
        apply_pair(o, sc, k * QR_PAIR, 0, 0, trans, s);
    }
    DD_HIP(hipStreamSynchronize(s));
}

// Q [I; 0] (the first C.n columns of Q) for C preset to the identity: the
// blocks are applied last to first, and each one only to the columns from its
// own first reflector on (the columns left of it are still unit vectors
// supported above the block's rows).
void orgqr_vb(Batch<ORItem>& o, hipStream_t s) {
    int kmax = 0;
    for (auto& x : o.h) kmax = std::max(kmax, std::min(x.V.n, x.V.m));
    QrScratch sc;
    sc.alloc(o.h, s);
    const int nb = ceil_div(kmax, QR_PAIR);
    for (int step = nb - 1; step >= 0; --step) apply_pair(o, sc, step * QR_PAIR, 3, 0, false, s);
    DD_HIP(hipStreamSynchronize(s));
}

// ===========================================================================
// Tridiagonalisation Q^T A Q = T (symmetric A, lower triangle), blocked in
// panels of TRD_NB columns: within a panel each column first receives the
// pending rank-2 updates of the panel's earlier columns, then yields its
// Householder vector v and w = tau (A22 v - V (W^T v) - W (V^T v)),
// w += -(tau/2)(w.v) v, with A22 not yet updated by the panel; after the
// panel the lower tiles of the trailing matrix take A22 -= V W^T + W V^T in
// one MFMA pass (K = 2 TRD_NB).  Every step reads the lower triangle only.
// Reflector k is stored in column k, rows k+2.., with an explicit 1 at row k+1.
// ===========================================================================
struct OpTrdCol {
    const TriItem* t;
    int k0, i;
    __device__ int tiles(int b) const { return t[b].A.n > k0 + i ? 1 : 0; }
    __device__ void operator()(int b, int) const {
        __shared__ double vk[TRD_NB], wk[TRD_NB];
        __shared__ double red[4];
        __shared__ double sc;
        const TriItem& T = t[b];
        const int n = T.A.n, ld = T.A.ld, k = k0 + i;
        double* A = T.A.p;
        if ((int)threadIdx.x < i) {
            const int j = threadIdx.x, c = k0 + j;
            vk[j] = (k == c + 1) ? 1.0 : A[k + (int64_t)c * ld];
            wk[j] = T.W[k + (int64_t)j * n];
        }
        __syncthreads();
        double* col = A + (int64_t)k * ld;
        for (int r = k + threadIdx.x; r < n; r += blockDim.x) {
            double a = col[r];
            for (int j = 0; j < i; ++j) {
                const int c = k0 + j;
                const double vr = (r == c + 1) ? 1.0 : A[r + (int64_t)c * ld];
                a -= vr * wk[j] + T.W[r + (int64_t)j * n] * vk[j];
            }
            col[r] = a;
        }
        __syncthreads();
        if (k == n - 1) {
            if (threadIdx.x == 0) T.d[k] = col[k];
            return;
        }
        double p = 0.0;
        for (int r = k + 2 + threadIdx.x; r < n; r += blockDim.x) p += col[r] * col[r];
        const double xn2 = block_sum(p, red);
        if (threadIdx.x == 0) {
            const double alpha = col[k + 1];
            double tau = 0.0, beta = alpha, scal = 0.0;
            if (xn2 > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            T.d[k] = col[k];
            T.e[k] = beta;
            T.tau[k] = tau;
            col[k + 1] = 1.0;
            sc = scal;
        }
        __syncthreads();
        const double scal = sc;
        for (int r = k + 2 + threadIdx.x; r < n; r += blockDim.x) col[r] *= scal;
    }
};

// y = A22 v from the lower triangle of A22.  A tile is a 64-column block J
// and a chunk of up to TRD_RB 64-row blocks I >= J below it; each 64 x 64
// block is staged in LDS (the next one's loads are in flight meanwhile) and
// adds A_IJ v_J to the rows of block I (row partial yp[J n + r]) and A_IJ^T
// v_I to the columns of block J, summed over the chunk (column partial
// yp[T n + (J T + chunk) 64 + c]); on diagonal blocks the stored diagonal
// counts once.  Extra tiles give the corrections t1_j = W(:, j)^T v,
// t2_j = V(:, j)^T v.
__host__ __device__ inline int trd_symv_tiles(int TL) {
    int n = 0;
    for (int J = 0; J < TL; ++J) n += (TL - J + TRD_RB - 1) / TRD_RB;
    return n;
}
struct OpTrdSymv {
    const TriItem* t;
    int k0, i;
    __device__ int tiles(int b) const {
        const int L = t[b].A.n - (k0 + i) - 1;
        return (L >= 1) ? trd_symv_tiles((L + 63) / 64) + i : 0;
    }
    __device__ void operator()(int b, int tile) const {
        __shared__ double As[64][65];
        __shared__ double vi[64], vj[64];
        __shared__ double red[2][4][64];
        const TriItem& T = t[b];
        const int n = T.A.n, ld = T.A.ld, k = k0 + i;
        const int L = n - k - 1;
        const double* v = T.A.p + (k + 1) + (int64_t)k * ld;  // v[0] = 1 stored
        const int TL = (L + 63) / 64;
        const int nsym = trd_symv_tiles(TL);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (tile < nsym) {
            int J = 0, ch = tile;
            for (;;) {
                const int c = (TL - J + TRD_RB - 1) / TRD_RB;
                if (ch < c) break;
                ch -= c;
                ++J;
            }
            const int Ib = J + ch * TRD_RB, Ie = min(TL, Ib + TRD_RB);
            const int j0 = J * 64;
            const double* A22 = T.A.p + (k + 1) + (int64_t)(k + 1) * ld;
            double cur[16];
            const int64_t ld4 = 4 * (int64_t)ld;
            auto fetch = [&](int I) {
                const int gr = I * 64 + lane;
                // columns gc = j0 + wv + 4 q < min(L, gr + 1)
                const int cend = (gr < L) ? gr + 1 - (j0 + wv) : 0;
                const double* p = A22 + gr + (int64_t)(j0 + wv) * ld;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    cur[q] = (4 * q < cend) ? *p : 0.0;
                    p += ld4;
                }
            };
            fetch(Ib);
            if (threadIdx.x < 64) vj[lane] = (j0 + lane < L) ? v[j0 + lane] : 0.0;
            double sc = 0.0;
            for (int I = Ib; I < Ie; ++I) {
                const int gr = I * 64 + lane;
#pragma unroll
                for (int q = 0; q < 16; ++q) As[wv + 4 * q][lane] = cur[q];
                if (threadIdx.x >= 64 && threadIdx.x < 128) vi[lane] = (gr < L) ? v[gr] : 0.0;
                __syncthreads();
                if (I + 1 < Ie) fetch(I + 1);
                // rows: lane = row, wave wv takes columns 16 wv .. 16 wv + 15
                double sr = 0.0;
#pragma unroll 4
                for (int q = 0; q < 16; ++q) sr += As[16 * wv + q][lane] * vj[16 * wv + q];
                // columns: lane = column, wave wv takes rows 16 wv .. 16 wv + 15
                // (the diagonal of a diagonal block is already in the row sums)
#pragma unroll 4
                for (int q = 0; q < 16; ++q) {
                    const int r = 16 * wv + q;
                    const double a = (I == J && r == lane) ? 0.0 : As[lane][r];
                    sc += a * vi[r];
                }
                red[0][wv][lane] = sr;
                __syncthreads();
                if (threadIdx.x < 64 && gr < L)
                    T.yp[(int64_t)J * n + gr] = (red[0][0][lane] + red[0][1][lane]) + (red[0][2][lane] + red[0][3][lane]);
            }
            red[1][wv][lane] = sc;
            __syncthreads();
            if (threadIdx.x < 64) {
                const int64_t Tn = (n + 63) / 64;
                T.yp[Tn * n + ((int64_t)J * Tn + ch) * 64 + lane] =
                    (red[1][0][lane] + red[1][1][lane]) + (red[1][2][lane] + red[1][3][lane]);
            }
            return;
        }
        const int j = tile - nsym;
        const double* wc = T.W + (k + 1) + (int64_t)j * n;
        const double* vc = T.A.p + (k + 1) + (int64_t)(k0 + j) * ld;  // rows > k0+j+1: stored values
        double s1 = 0.0, s2 = 0.0;
        for (int r = threadIdx.x; r < L; r += blockDim.x) {
            const double vr = v[r];
            s1 += wc[r] * vr;
            s2 += vc[r] * vr;
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        double (*r2)[4] = reinterpret_cast<double (*)[4]>(&red[0][0][0]);
        if (lane == 0) { r2[0][wv] = s1; r2[1][wv] = s2; }
        __syncthreads();
        if (threadIdx.x == 0) {
            T.aux[j] = (r2[0][0] + r2[0][1]) + (r2[0][2] + r2[0][3]);
            T.aux[TRD_NB + j] = (r2[1][0] + r2[1][1]) + (r2[1][2] + r2[1][3]);
        }
    }
};

// w = tau (y - V t1 - W t2) into column i of W; partial sums of w.v
struct OpTrdW {
    const TriItem* t;
    int k0, i;
    __device__ int tiles(int b) const {
        const int L = t[b].A.n - (k0 + i) - 1;
        return (L >= 1) ? (L + 255) / 256 : 0;
    }
    __device__ void operator()(int b, int tile) const {
        __shared__ double red[4];
        const TriItem& T = t[b];
        const int n = T.A.n, ld = T.A.ld, k = k0 + i;
        const int L = n - k - 1;
        const double tau = T.tau[k];
        const int r = tile * 256 + threadIdx.x;
        double pv = 0.0;
        if (r < L) {
            const int g = k + 1 + r;
            // y_r: row partials of blocks J <= r/64, column partials of the
            // row chunks below column block r/64
            const int64_t Tn = (n + 63) / 64;
            const int Jr = r >> 6, TL = (L + 63) / 64;
            const int nch = (TL - Jr + TRD_RB - 1) / TRD_RB;
            double y0 = 0.0, y1 = 0.0;
            for (int J = 0; J <= Jr; ++J) y0 += T.yp[(int64_t)J * n + r];
            const double* pc = T.yp + Tn * n + (int64_t)Jr * Tn * 64 + (r & 63);
            for (int c = 0; c < nch; ++c) y1 += pc[(int64_t)c * 64];
            double w = y0 + y1;
            for (int j = 0; j < i; ++j)
                w -= T.A.p[g + (int64_t)(k0 + j) * ld] * T.aux[j] + T.W[g + (int64_t)j * n] * T.aux[TRD_NB + j];
            w *= tau;
            T.W[g + (int64_t)i * n] = w;
            pv = w * T.A.p[g + (int64_t)k * ld];
        }
        pv = block_sum(pv, red);
        if (threadIdx.x == 0) T.part[tile] = pv;
    }
};

// w += -(tau/2)(w.v) v
struct OpTrdAlpha {
    const TriItem* t;
    int k0, i;
    __device__ int tiles(int b) const {
        const int L = t[b].A.n - (k0 + i) - 1;
        return (L >= 1) ? (L + 255) / 256 : 0;
    }
    __device__ void operator()(int b, int tile) const {
        const TriItem& T = t[b];
        const int n = T.A.n, ld = T.A.ld, k = k0 + i;
        const int L = n - k - 1;
        const int nt = (L + 255) / 256;
        double s = 0.0;
        for (int q = 0; q < nt; ++q) s += T.part[q];
        const double alpha = -0.5 * T.tau[k] * s;
        const int r = tile * 256 + threadIdx.x;
        if (r < L) {
            const int g = k + 1 + r;
            T.W[g + (int64_t)i * n] += alpha * T.A.p[g + (int64_t)k * ld];
        }
    }
};

// lower tiles of C += alpha (A B^T + B A^T), A and B M x K (column-major):
// both products accumulate in one tile, then one read-modify-write of C
struct OpSyr2kLower {
    const GemmItem* g;
    __device__ int tiles(int b) const {
        const int T = (g[b].M + 63) / 64;
        return T * (T + 1) / 2;
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemC sm;
        const GemmItem& G = g[b];
        int tj = 0, r = t;
        const int T = (G.M + 63) / 64;
        while (r >= T - tj) {
            r -= T - tj;
            ++tj;
        }
        const int ti = tj + r;
        const int i0 = ti * 64, j0 = tj * 64;
        double4_t acc[2][2];
        acc_zero(acc);
        mfma_tile_64<false, true>(G.A, G.lda, G.B, G.ldb, G.M, G.M, G.K, i0, j0, sm.t, acc);
        mfma_tile_64<false, true>(G.B, G.ldb, G.A, G.lda, G.M, G.M, G.K, i0, j0, sm.t, acc);
        double* C = G.C;
        const int ldc = G.ldc, M = G.M;
        const double al = G.alpha;
        acc_store_coalesced(acc, sm, [&](int rr, int c, double v) {
            const int gi = i0 + rr, gj = j0 + c;
            if (gi < M && gj < M) C[gi + (int64_t)gj * ldc] += al * v;
        });
    }
};

void sytrd_vb(Batch<TriItem>& t, hipStream_t s) {
    int nmax = 0;
    for (auto& x : t.h) nmax = std::max(nmax, x.A.n);
    for (int k0 = 0; k0 < nmax; k0 += TRD_NB) {
        for (int i = 0; i < TRD_NB && k0 + i < nmax; ++i) {
            const int k = k0 + i;
            int64_t nc = 0, ns = 0, nw = 0;
            for (auto& x : t.h) {
                if (x.A.n <= k) continue;
                ++nc;
                const int L = x.A.n - k - 1;
                if (L >= 1) {
                    ns += trd_symv_tiles(ceil_div(L, 64)) + i;
                    nw += ceil_div(L, 256);
                }
            }
            launch_tiles(OpTrdCol{t.d.p, k0, i}, t.size(), nc, s, "trd_col");
            if (ns) {
                launch_tiles(OpTrdSymv{t.d.p, k0, i}, t.size(), ns, s, "trd_symv");
                launch_tiles(OpTrdW{t.d.p, k0, i}, t.size(), nw, s, "trd_w");
                launch_tiles(OpTrdAlpha{t.d.p, k0, i}, t.size(), nw, s, "trd_alpha");
            }
        }
        // trailing update A22 -= V W^T + W V^T, lower tiles (rows/columns from k0 + TRD_NB)
        const int k1 = k0 + TRD_NB;
        Batch<GemmItem> g1;
        int64_t nt = 0;
        for (auto& x : t.h) {
            const int m = x.A.n - k1;
            if (m <= 0) continue;
            double* C = x.A.p + k1 + (int64_t)k1 * x.A.ld;
            const double* V = x.A.p + k1 + (int64_t)k0 * x.A.ld;
            const double* Wm = x.W + k1;
            g1.h.push_back(GemmItem{V, x.A.ld, Wm, x.A.n, C, x.A.ld, m, m, TRD_NB, -1.0, 1.0});
            const int64_t T = ceil_div(m, 64);
            nt += T * (T + 1) / 2;
        }
        if (!g1.h.empty()) {
            g1.sync(s);
            launch_tiles(OpSyr2kLower{g1.d.p}, g1.size(), nt, s, "trd_syr2k");
            DD_HIP(hipStreamSynchronize(s));  // the host batch is freed at scope exit
        }
    }
}

// ===========================================================================
// Bisection on the symmetric tridiagonal (Sturm counts)
// ===========================================================================
__device__ int sturm_count(const double* d, const double* e, int n, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
        q = d[i] - x - e[i - 1] * e[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// Gershgorin interval, pivmin and the number of eigenvalues below the
// threshold (capped), one thread per item: aux[3b..3b+2] = (gl, gu, pivmin).
struct OpStebzCount {
    const EigItem* it;
    double* aux;
    __device__ int tiles(int b) const { return 1; }
    __device__ void operator()(int b, int) const {
        const EigItem& E = it[b];
        const int n = E.n;
        if (threadIdx.x != 0) return;
        if (n <= 0) {
            *E.count = 0;
            return;
        }
        double lo = 1e300, hi = -1e300, emax = 0.0;
        for (int i = 0; i < n; ++i) {
            const double r = (i > 0 ? fabs(E.e[i - 1]) : 0.0) + (i < n - 1 ? fabs(E.e[i]) : 0.0);
            lo = fmin(lo, E.d[i] - r);
            hi = fmax(hi, E.d[i] + r);
            if (i < n - 1) emax = fmax(emax, E.e[i] * E.e[i]);
        }
        const double nrm = fmax(fabs(lo), fabs(hi));
        const double pivmin = fmax(2.2250738585072014e-308, 2.2250738585072014e-308 * emax) * 4.0;
        aux[3 * b] = lo - 2.0 * nrm * 2.220446049250313e-16 * n - pivmin;
        aux[3 * b + 1] = hi + 2.0 * nrm * 2.220446049250313e-16 * n + pivmin;
        aux[3 * b + 2] = pivmin;
        *E.count = min(sturm_count(E.d, E.e, n, E.thr, pivmin), E.cap);
    }
};

// j-th smallest eigenvalue = smallest x with count(x) >= j + 1, by 4-point
// multisection: four lanes evaluate the Sturm count at the interior points
// of a 5-way split of [lo, hi] and the interval shrinks to the sub-interval
// where the count first reaches j + 1.  The stopping test is that of plain
// bisection (width <= 2 eps max(|lo|, |hi|) + pivmin).  A tile is 64
// eigenvalues; d and e^2 are staged in LDS when they fit.
constexpr int STEBZ_LDS = 4096;  // doubles per array staged in LDS
struct OpStebzBisect {
    const EigItem* it;
    const double* aux;
    __device__ int tiles(int b) const { return (min(it[b].n, it[b].cap) + 63) / 64; }
    __device__ void operator()(int b, int t) const {
        __shared__ double ds[STEBZ_LDS], e2s[STEBZ_LDS];
        const EigItem& E = it[b];
        const int n = E.n;
        const int cnt = *E.count;
        if (t * 64 >= cnt) return;
        const bool inl = n <= STEBZ_LDS;
        if (inl) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                ds[i] = E.d[i];
                e2s[i] = (i < n - 1) ? E.e[i] * E.e[i] : 0.0;
            }
        }
        __syncthreads();
        const double* d = inl ? ds : E.d;
        const double gl = aux[3 * b], gu = aux[3 * b + 1], pivmin = aux[3 * b + 2];
        const double eps = 2.220446049250313e-16;
        const int lane = threadIdx.x & 63, sub = lane & 3;
        const int j = t * 64 + (int)(threadIdx.x >> 2);
        const bool active = j < cnt;  // uniform over the 4 lanes of an eigenvalue
        double lo = gl, hi = fmin(gu, E.thr);
        for (int itn = 0; itn < 200; ++itn) {
            const bool done = !active || (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin);
            if (__all(done)) break;
            const double h = (hi - lo) * 0.2;
            const double x = lo + (sub + 1) * h;
            int c = 0;
            if (!done) {
                double q = d[0] - x;
                if (fabs(q) < pivmin) q = -pivmin;
                if (q < 0) ++c;
                if (inl) {
                    for (int i = 1; i < n; ++i) {
                        q = d[i] - x - e2s[i - 1] / q;
                        if (fabs(q) < pivmin) q = -pivmin;
                        if (q < 0) ++c;
                    }
                } else {
                    for (int i = 1; i < n; ++i) {
                        q = d[i] - x - E.e[i - 1] * E.e[i - 1] / q;
                        if (fabs(q) < pivmin) q = -pivmin;
                        if (q < 0) ++c;
                    }
                }
            }
            // flags of the 4 points of this eigenvalue: bit k = count(x_k) >= j + 1
            const int f = (c >= j + 1) ? 1 : 0;
            const int base = lane & ~3;
            const int f0 = __shfl(f, base, 64), f1 = __shfl(f, base + 1, 64);
            const int f2 = __shfl(f, base + 2, 64), f3 = __shfl(f, base + 3, 64);
            if (!done) {
                // first point whose count reaches j + 1 (4 if none)
                const int k = f0 ? 0 : (f1 ? 1 : (f2 ? 2 : (f3 ? 3 : 4)));
                const double nlo = (k == 0) ? lo : lo + k * h;
                const double nhi = (k == 4) ? hi : lo + (k + 1) * h;
                lo = nlo;
                hi = nhi;
            }
        }
        if (active && sub == 0) E.mu[j] = 0.5 * (lo + hi);
    }
};

void stebz_vb(Batch<EigItem>& e, hipStream_t s) {
    DBuf<double> aux(3 * std::max(1, e.size()));
    int64_t nt = 0;
    for (auto& x : e.h) nt += ceil_div(std::min(x.n, x.cap), 64);
    launch_tiles(OpStebzCount{e.d.p, aux.p}, e.size(), e.size(), s, "stebz_count");
    if (nt) launch_tiles(OpStebzBisect{e.d.p, aux.p}, e.size(), nt, s, "stebz");
    DD_HIP(hipStreamSynchronize(s));  // aux is freed on return
}

// ===========================================================================
// Inverse iteration on the tridiagonal (T - mu I) x = y, LU with partial
// pivoting (one thread per system), clusters orthogonalised by the block.
// ===========================================================================
__device__ unsigned int hash_u32(unsigned int x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

// Solve (T - mu I) x = y in place by Gaussian elimination with partial
// pivoting on the tridiagonal (the working row carries two entries; a row
// swap gives U a second superdiagonal).  Zero pivots are replaced by `tiny`.
// Work arrays and x are strided (element i at [i * st]) so that the threads of
// a wave, each solving its own system, touch consecutive addresses.
__device__ void tri_solve(const double* d, const double* e, int n, double mu, double* u1, double* u2, double* u3,
                          double* x, int st, double tiny) {
    double a = d[0] - mu;
    double bb = (n > 1) ? e[0] : 0.0;
    double xi = x[0];
    for (int i = 0; i < n - 1; ++i) {
        const double c = e[i];
        const double dn = d[i + 1] - mu;
        const double en = (i + 1 < n - 1) ? e[i + 1] : 0.0;
        const double xn = x[(int64_t)(i + 1) * st];
        if (fabs(a) >= fabs(c)) {
            if (a == 0.0) a = tiny;
            const double m = c / a;
            u1[(int64_t)i * st] = a; u2[(int64_t)i * st] = bb; u3[(int64_t)i * st] = 0.0;
            x[(int64_t)i * st] = xi;
            xi = xn - m * xi;
            a = dn - m * bb;
            bb = en;
        } else {
            const double m = a / c;
            u1[(int64_t)i * st] = c; u2[(int64_t)i * st] = dn; u3[(int64_t)i * st] = en;
            x[(int64_t)i * st] = xn;
            xi = xi - m * xn;
            a = bb - m * dn;
            bb = -m * en;
        }
    }
    if (a == 0.0) a = tiny;
    u1[(int64_t)(n - 1) * st] = a;
    double x1 = xi / a;  // x[n-1]
    x[(int64_t)(n - 1) * st] = x1;
    if (n > 1) {
        double x0 = (x[(int64_t)(n - 2) * st] - u2[(int64_t)(n - 2) * st] * x1) / u1[(int64_t)(n - 2) * st];
        x[(int64_t)(n - 2) * st] = x0;
        for (int i = n - 3; i >= 0; --i) {
            const double v = (x[(int64_t)i * st] - u2[(int64_t)i * st] * x0 - u3[(int64_t)i * st] * x1) / u1[(int64_t)i * st];
            x[(int64_t)i * st] = v;
            x1 = x0;
            x0 = v;
        }
    }
}

__device__ double start_value(int i, int j) {
    return 1.0 + 0.5 * ((hash_u32((unsigned)i * 2654435761u + (unsigned)j * 40503u + 12345u) & 0xffff) / 65536.0 - 0.5);
}

// One inverse-iteration round for every eigenvalue of the item (one thread per
// eigenvalue, the block's 256 threads sweep the list): x_j <- (T - mu_j I)^{-1} x_j,
// normalised.  first: start from the hashed vector instead of Y.
struct OpSteinSolve {
    const VecItem* it;
    int first;
    // 256 eigenvectors per workgroup, each workgroup with its own work arrays
    __device__ int tiles(int b) const { return it[b].n > 0 ? (*it[b].count + 255) / 256 : 0; }
    __device__ void operator()(int b, int tile) const {
        __shared__ int s_cnt;
        __shared__ double s_tn;
        const VecItem& V = it[b];
        const int n = V.n;
        if (threadIdx.x == 0) {
            s_cnt = *V.count;
            double tn = 0.0;
            for (int i = 0; i < n; ++i)
                tn = fmax(tn, fabs(V.d[i]) + (i > 0 ? fabs(V.e[i - 1]) : 0.0) + (i < n - 1 ? fabs(V.e[i]) : 0.0));
            s_tn = fmax(tn, 1e-300);
        }
        __syncthreads();
        const int p = s_cnt;
        const double tiny = 2.220446049250313e-16 * s_tn;
        const int t = threadIdx.x;
        double* u1 = V.work + (int64_t)tile * 4 * n * 256 + t;
        double* u2 = u1 + (int64_t)n * 256;
        double* u3 = u2 + (int64_t)n * 256;
        double* x = u3 + (int64_t)n * 256;
        {
            const int j = tile * 256 + t;
            if (j >= p) return;
            double* y = V.Y + (int64_t)j * V.ldy;
            for (int i = 0; i < n; ++i) x[(int64_t)i * 256] = first ? start_value(i, j) : y[i];
            tri_solve(V.d, V.e, n, V.mu[j], u1, u2, u3, x, 256, tiny);
            double nr = 0.0;
            for (int i = 0; i < n; ++i) nr += x[(int64_t)i * 256] * x[(int64_t)i * 256];
            nr = 1.0 / sqrt(nr);
            for (int i = 0; i < n; ++i) y[i] = x[(int64_t)i * 256] * nr;
        }
    }
};

void stein_vb(Batch<VecItem>& v, const std::vector<std::vector<double>>& hmu, double cluster_tol, hipStream_t s) {
    // clusters (size >= 2) become the items of a batched Householder QR
    Batch<QRItem> qb;
    Batch<ORItem> ob;
    std::vector<int64_t> sz_q, sz_T, sz_W, sz_t;
    struct Cl { int item, c0, c; };
    std::vector<Cl> cls;
    for (int b = 0; b < v.size(); ++b) {
        const auto& mu = hmu[b];
        const int p = (int)mu.size();
        double tn = 0.0;
        for (double m : mu) tn = std::max(tn, std::fabs(m));
        const double gap = cluster_tol * std::max(1.0, tn);
        int c0 = 0;
        for (int j = 1; j <= p; ++j) {
            if (j == p || mu[j] - mu[j - 1] > gap) {
                if (j - c0 >= 2) cls.push_back(Cl{b, c0, j - c0});
                c0 = j;
            }
        }
    }
    DBuf<double> tq, tT, tW, tQ, tG;
    std::vector<DMat> hsrc, hdst;
    if (!cls.empty()) {
        int64_t a = 0, bT = 0, bW = 0, bQ = 0, bG = 0;
        for (auto& c : cls) {
            const int n = v.h[c.item].n;
            a += c.c;
            bT += qr_t_size(c.c);
            bW += qr_w_size(c.c);
            bQ += (int64_t)n * c.c;
            bG += qr_g_size(c.c);
        }
        tq.alloc(a); tT.alloc(bT); tW.alloc(bW); tQ.alloc(bQ); tG.alloc(bG);
        a = bT = bW = bQ = bG = 0;
        for (auto& c : cls) {
            const VecItem& it = v.h[c.item];
            const int n = it.n;
            DMat Yc{it.Y + (int64_t)c.c0 * it.ldy, it.ldy, n, c.c};
            DMat Qc{tQ.p + bQ, n, n, c.c};
            qb.h.push_back(QRItem{Yc, tq.p + a, tT.p + bT, tW.p + bW, QR_NB, c.c, tG.p + bG});
            ob.h.push_back(ORItem{Yc, tT.p + bT, Qc, tW.p + bW, tG.p + bG});
            hsrc.push_back(Qc);
            hdst.push_back(Yc);
            a += c.c;
            bT += qr_t_size(c.c);
            bW += qr_w_size(c.c);
            bQ += (int64_t)n * c.c;
            bG += qr_g_size(c.c);
        }
        qb.sync(s);
        ob.sync(s);
    }
    Batch<DMat> Qs, Ys;
    Qs.h = hsrc;
    Ys.h = hdst;
    if (!cls.empty()) { Qs.sync(s); Ys.sync(s); }
    int64_t nst = 0;
    for (int b = 0; b < v.size(); ++b) nst += ceil_div((int64_t)hmu[b].size(), 256);
    for (int round = 0; round < 3; ++round) {
        launch_tiles(OpSteinSolve{v.d.p, round == 0}, v.size(), nst, s, "stein_solve");
        if (!cls.empty()) {
            geqrf_vb(qb, s);
            set_identity_vb(Qs, 1.0, s);
            orgqr_vb(ob, s);
            copy_vb(Qs, Ys, false, 1.0, s);
        }
    }
    DD_HIP(hipStreamSynchronize(s));
}

// ===========================================================================
// elementwise helpers
// ===========================================================================
struct OpSetId {
    const DMat* A;
    double dg;
    __device__ int tiles(int b) const { return (int)(((int64_t)A[b].m * A[b].n + 16383) / 16384); }
    __device__ void operator()(int b, int t) const {
        const DMat M = A[b];
        const int64_t tot = (int64_t)M.m * M.n;
        for (int64_t e = (int64_t)t * 16384 + threadIdx.x; e < min(tot, (int64_t)(t + 1) * 16384); e += blockDim.x) {
            const int r = (int)(e % M.m), c = (int)(e / M.m);
            M.p[r + (int64_t)c * M.ld] = (r == c) ? dg : 0.0;
        }
    }
};
void set_identity_vb(Batch<DMat>& A, double diag, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : A.h) tot += ((int64_t)x.m * x.n + 16383) / 16384;
    launch_tiles(OpSetId{A.d.p, diag}, A.size(), tot, s, "set_identity");
}

struct OpCopy {
    const DMat* S;
    const DMat* D;
    bool tr;
    double sc;
    __device__ int tiles(int b) const { return ((D[b].m + 63) / 64) * ((D[b].n + 63) / 64); }
    __device__ void operator()(int b, int t) const {
        __shared__ double tile[64][65];
        const DMat s = S[b], d = D[b];
        const int tm = (d.m + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        if (!tr) {
            for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
                const int r = i0 + (e & 63), c = j0 + (e >> 6);
                if (r < d.m && c < d.n) d.p[r + (int64_t)c * d.ld] = sc * s.p[r + (int64_t)c * s.ld];
            }
        } else {
            // d(r, c) = s(c, r)
            for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
                const int cc = e & 63, rr = e >> 6;  // read s rows j0+cc, cols i0+rr (coalesced in cc)
                const int sr = j0 + cc, scol = i0 + rr;
                tile[rr][cc] = (sr < d.n && scol < d.m) ? s.p[sr + (int64_t)scol * s.ld] : 0.0;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
                const int r = e & 63, c = e >> 6;
                if (i0 + r < d.m && j0 + c < d.n) d.p[(i0 + r) + (int64_t)(j0 + c) * d.ld] = sc * tile[r][c];
            }
        }
    }
};
// S (2n x n) = [sc X^T; I] interleaved by rows: 64 x 64 tiles of (i, j), X^T
// read through LDS as in the transposed copy
struct OpStackInterleaved {
    const DMat* X;
    const DMat* S;
    const double* sc;
    __device__ int tiles(int b) const { return ((X[b].n + 63) / 64) * ((X[b].n + 63) / 64); }
    __device__ void operator()(int b, int t) const {
        __shared__ double tile[64][65];
        const DMat x = X[b], d = S[b];
        const int n = x.n, T = (n + 63) / 64;
        const int i0 = (t % T) * 64, j0 = (t / T) * 64;
        for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
            const int cc = e & 63, rr = e >> 6;  // X(j0 + cc, i0 + rr), coalesced in cc
            tile[rr][cc] = (j0 + cc < n && i0 + rr < n) ? x.p[(j0 + cc) + (int64_t)(i0 + rr) * x.ld] : 0.0;
        }
        __syncthreads();
        const double a = sc[b];
        for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
            const int r = e & 63, c = e >> 6, i = i0 + r, j = j0 + c;
            if (i < n && j < n) {
                d.p[2 * i + (int64_t)j * d.ld] = a * tile[r][c];
                d.p[2 * i + 1 + (int64_t)j * d.ld] = i == j ? 1.0 : 0.0;
            }
        }
    }
};
void stack_interleaved_vb(Batch<DMat>& X, Batch<DMat>& S, const double* dscale, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : X.h) tot += (int64_t)ceil_div(x.n, 64) * ceil_div(x.n, 64);
    launch_tiles(OpStackInterleaved{X.d.p, S.d.p, dscale}, X.size(), tot, s, "stack_interleaved");
}

// D[i] = Q[2i], D[n + i] = Q[2i + 1] (rows), 256 rows of D per tile and column
struct OpDeinterleave {
    const DMat* Q;
    const DMat* D;
    __device__ int tiles(int b) const { return ((D[b].m + 255) / 256) * D[b].n; }
    __device__ void operator()(int b, int t) const {
        const DMat q = Q[b], d = D[b];
        const int nb = (d.m + 255) / 256, h = d.m / 2;
        const int j = t / nb, r = (t % nb) * 256 + threadIdx.x;
        if (r < d.m) d.p[r + (int64_t)j * d.ld] = q.p[(r < h ? 2 * r : 2 * (r - h) + 1) + (int64_t)j * q.ld];
    }
};
void deinterleave_rows_vb(Batch<DMat>& Q, Batch<DMat>& D, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : D.h) tot += (int64_t)ceil_div(x.m, 256) * x.n;
    launch_tiles(OpDeinterleave{Q.d.p, D.d.p}, D.size(), tot, s, "deinterleave");
}

void copy_vb(Batch<DMat>& src, Batch<DMat>& dst, bool transpose, double scale, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : dst.h) tot += (int64_t)ceil_div(x.m, 64) * ceil_div(x.n, 64);
    launch_tiles(OpCopy{src.d.p, dst.d.p, transpose, scale}, dst.size(), tot, s, "copy");
}

struct OpAddDiag {
    const DMat* A;
    const double* sh;
    __device__ int tiles(int b) const { return (A[b].n + 255) / 256; }
    __device__ void operator()(int b, int t) const {
        const int i = t * 256 + threadIdx.x;
        if (i < A[b].n && i < A[b].m) A[b].p[i + (int64_t)i * A[b].ld] += sh[b];
    }
};
void add_diag_vb(Batch<DMat>& A, const double* dshift, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : A.h) tot += ceil_div(x.n, 256);
    launch_tiles(OpAddDiag{A.d.p, dshift}, A.size(), tot, s, "add_diag");
}

struct OpSym {
    const DMat* A;
    __device__ int tiles(int b) const { const int T = (A[b].n + 63) / 64; return T * (T + 1) / 2; }
    __device__ void operator()(int b, int t) const {
        const DMat M = A[b];
        int ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        const int tj = t - ti * (ti + 1) / 2;
        for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
            const int r = ti * 64 + (e & 63), c = tj * 64 + (e >> 6);
            if (r < M.n && c < M.n && r > c) {
                double* a = M.p + r + (int64_t)c * M.ld;
                double* bq = M.p + c + (int64_t)r * M.ld;
                const double v = 0.5 * (*a + *bq);
                *a = v;
                *bq = v;
            }
        }
    }
};
void symmetrize_vb(Batch<DMat>& A, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : A.h) { const int T = ceil_div(x.n, 64); tot += (int64_t)T * (T + 1) / 2; }
    launch_tiles(OpSym{A.d.p}, A.size(), tot, s, "symmetrize");
}

struct OpZeroUpper {
    const DMat* A;
    __device__ int tiles(int b) const { return ((A[b].m + 63) / 64) * ((A[b].n + 63) / 64); }
    __device__ void operator()(int b, int t) const {
        const DMat M = A[b];
        const int tm = (M.m + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
            const int r = i0 + (e & 63), c = j0 + (e >> 6);
            if (r < M.m && c < M.n && r < c) M.p[r + (int64_t)c * M.ld] = 0.0;
        }
    }
};
void zero_upper_vb(Batch<DMat>& A, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : A.h) tot += (int64_t)ceil_div(x.m, 64) * ceil_div(x.n, 64);
    launch_tiles(OpZeroUpper{A.d.p}, A.size(), tot, s, "zero_upper");
}

struct OpZeroLower {
    const DMat* A;
    __device__ int tiles(int b) const { return ((A[b].m + 63) / 64) * ((A[b].n + 63) / 64); }
    __device__ void operator()(int b, int t) const {
        const DMat M = A[b];
        const int tm = (M.m + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
            const int r = i0 + (e & 63), c = j0 + (e >> 6);
            if (r < M.m && c < M.n && r > c) M.p[r + (int64_t)c * M.ld] = 0.0;
        }
    }
};
void zero_lower_vb(Batch<DMat>& A, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : A.h) tot += (int64_t)ceil_div(x.m, 64) * ceil_div(x.n, 64);
    launch_tiles(OpZeroLower{A.d.p}, A.size(), tot, s, "zero_lower");
}

struct OpAxpby {
    const DMat* X;
    const DMat* Y;
    const double* al;
    const double* be;
    __device__ int tiles(int b) const { return ((Y[b].m + 63) / 64) * ((Y[b].n + 63) / 64); }
    __device__ void operator()(int b, int t) const {
        const DMat x = X[b], y = Y[b];
        const int tm = (y.m + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        const double a = al[b], c = be[b];
        for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
            const int r = i0 + (e & 63), cc = j0 + (e >> 6);
            if (r < y.m && cc < y.n) {
                double* py = y.p + r + (int64_t)cc * y.ld;
                *py = a * x.p[r + (int64_t)cc * x.ld] + c * *py;
            }
        }
    }
};
void axpby_vb(Batch<DMat>& X, Batch<DMat>& Y, const double* dalpha, const double* dbeta, hipStream_t s) {
    int64_t tot = 0;
    for (auto& x : Y.h) tot += (int64_t)ceil_div(x.m, 64) * ceil_div(x.n, 64);
    launch_tiles(OpAxpby{X.d.p, Y.d.p, dalpha, dbeta}, Y.size(), tot, s, "axpby");
}

// ||A||_F: partial sums over 16-column slabs, then an ordered sum per item
struct OpFrobPart {
    const DMat* A;
    double* const* part;
    __device__ int tiles(int b) const { return (A[b].n + 15) / 16; }
    __device__ void operator()(int b, int t) const {
        __shared__ double red[4];
        const DMat M = A[b];
        double s = 0.0;
        for (int c = t * 16; c < min(M.n, t * 16 + 16); ++c)
            for (int r = threadIdx.x; r < M.m; r += blockDim.x) {
                const double v = M.p[r + (int64_t)c * M.ld];
                s += v * v;
            }
        s = block_sum(s, red);
        if (threadIdx.x == 0) part[b][t] = s;
    }
};
struct OpFrob {
    const DMat* A;
    double* const* part;
    double* out;
    __device__ int tiles(int b) const { return 1; }
    __device__ void operator()(int b, int) const {
        if (threadIdx.x != 0) return;
        double s = 0.0;
        for (int t = 0; t < (A[b].n + 15) / 16; ++t) s += part[b][t];
        out[b] = sqrt(s);
    }
};
void frob_vb(Batch<DMat>& A, double* dout, hipStream_t s) {
    std::vector<int64_t> off(A.size() + 1, 0);
    for (int b = 0; b < A.size(); ++b) off[b + 1] = off[b] + ceil_div(std::max(1, A.h[b].n), 16);
    DBuf<double> pbuf(std::max<int64_t>(1, off.back()));
    std::vector<double*> hp(A.size());
    for (int b = 0; b < A.size(); ++b) hp[b] = pbuf.p + off[b];
    DBuf<double*> dp(std::max<size_t>(1, hp.size()));
    h2d(dp.p, hp.data(), hp.size(), s);
    launch_tiles(OpFrobPart{A.d.p, dp.p}, A.size(), off.back(), s, "frob_part");
    launch_tiles(OpFrob{A.d.p, dp.p, dout}, A.size(), A.size(), s, "frob");
    DD_HIP(hipStreamSynchronize(s));
}

// Largest eigenvalue of the symmetric tridiagonal (a, b) of size m by bisection.
__device__ double tri_max_eig(const double* a, const double* b, int m) {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < m - 1 ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    const double pivmin = 1e-290;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi))) break;
        if (sturm_count(a, b, m, mid, pivmin) >= m) hi = mid;  // all eigenvalues below mid
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Lanczos state per item: V (n x (K+1)), w (n), al/be (K+1), step/done flags.
struct LzItem {
    DMat H;
    double* V;
    double* w;
    double* al;
    double* be;
    int* done;
    double* theta;
};

// w = H v_j, 64 rows per workgroup (H symmetric: w_r = H[:, r] . v_j, coalesced columns)
struct OpLzMatvec {
    const LzItem* it;
    int j;
    __device__ int tiles(int b) const { return (*it[b].done || j >= it[b].H.n) ? 0 : (it[b].H.n + 63) / 64; }
    __device__ void operator()(int b, int t) const {
        const LzItem& L = it[b];
        const int n = L.H.n;
        const double* v = L.V + (int64_t)j * n;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int rr = wv; rr < 64; rr += 4) {
            const int r = t * 64 + rr;
            if (r >= n) break;
            const double* col = L.H.p + (int64_t)r * L.H.ld;
            double sum = 0.0;
            for (int c = lane; c < n; c += 64) sum += col[c] * v[c];
            sum = wave_sum(sum);
            if (lane == 0) L.w[r] = sum;
        }
    }
};

// Full reorthogonalisation of w against v_0..v_j by classical Gram-Schmidt
// applied twice: h = V^T w (OpLzDots, 16 columns per workgroup), then
// w -= V h (OpLzUpd, 256 rows per workgroup); hp holds 2 (K+1) doubles per
// item, the dots of the two passes.
struct OpLzDots {
    const LzItem* it;
    double* const* hp;
    int j, K, pass;
    __device__ int tiles(int b) const { return (*it[b].done || j >= it[b].H.n) ? 0 : (j + 16) / 16; }
    __device__ void operator()(int b, int t) const {
        const LzItem& L = it[b];
        const int n = L.H.n;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int i0 = t * 16 + wv * 4;
        if (i0 > j) return;
        const int ni = min(4, j + 1 - i0);
        const double* V = L.V + (int64_t)i0 * n;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r = lane; r < n; r += 64) {
            const double wr = L.w[r];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (q < ni) a[q] += V[r + (int64_t)q * n] * wr;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = wave_sum(a[q]);
            if (lane == 0 && q < ni) hp[b][pass * (K + 1) + i0 + q] = v;
        }
    }
};
struct OpLzUpd {
    const LzItem* it;
    double* const* hp;
    int j, K, pass;
    __device__ int tiles(int b) const { return (*it[b].done || j >= it[b].H.n) ? 0 : (it[b].H.n + 255) / 256; }
    __device__ void operator()(int b, int t) const {
        const LzItem& L = it[b];
        const int n = L.H.n;
        const int r = t * 256 + threadIdx.x;
        if (r >= n) return;
        const double* h = hp[b] + pass * (K + 1);
        double a0 = 0.0, a1 = 0.0;
        int i = 0;
        for (; i + 1 <= j; i += 2) {
            a0 += L.V[r + (int64_t)i * n] * h[i];
            a1 += L.V[r + (int64_t)(i + 1) * n] * h[i + 1];
        }
        for (; i <= j; ++i) a0 += L.V[r + (int64_t)i * n] * h[i];
        L.w[r] -= a0 + a1;
    }
};
// alpha_j (both passes), beta_j = ||w||, v_{j+1} = w / beta_j, and the
// convergence test on the largest Ritz value every 4 steps.
struct OpLzFinish {
    const LzItem* it;
    double* const* hp;
    int j, K;
    __device__ int tiles(int b) const { return (*it[b].done || j >= it[b].H.n) ? 0 : 1; }
    __device__ void operator()(int b, int) const {
        __shared__ double red[4];
        __shared__ int s_stop;
        const LzItem& L = it[b];
        const int n = L.H.n;
        double* w = L.w;
        double nr = 0.0;
        for (int r = threadIdx.x; r < n; r += blockDim.x) nr += w[r] * w[r];
        nr = sqrt(block_sum(nr, red));
        if (threadIdx.x == 0) {
            L.al[j] = hp[b][j] + hp[b][(K + 1) + j];
            L.be[j] = nr;
            s_stop = 0;
            const bool last = (j + 1 >= min(K, n)) || nr == 0.0;
            if ((j % 4 == 3) || last) {
                const double th = tri_max_eig(L.al, L.be, j + 1);
                if (last || fabs(th - *L.theta) <= 1e-13 * fabs(th) || nr <= 1e-14 * fabs(th)) s_stop = 1;
                *L.theta = th;
            }
            if (s_stop) *L.done = 1;
        }
        __syncthreads();
        if (s_stop) return;
        double* vn = L.V + (int64_t)(j + 1) * n;
        for (int r = threadIdx.x; r < n; r += blockDim.x) vn[r] = w[r] / nr;
    }
};
__global__ void k_lz_init(LzItem* it, int nitems) {
    const int b = blockIdx.x;
    if (b >= nitems) return;
    const LzItem& L = it[b];
    const int n = L.H.n;
    for (int r = threadIdx.x; r < n; r += blockDim.x) L.V[r] = 1.0 / sqrt((double)n);
    if (threadIdx.x == 0) {
        *L.done = 0;
        *L.theta = 0.0;
    }
}

void lanczos_max_vb(Batch<DMat>& H, double* const* work, int K, double* dout, int* dsteps, hipStream_t s) {
    const int N = H.size();
    K = std::min(K, 128);
    Batch<LzItem> lz;
    std::vector<double*> hw(N);
    DD_HIP(hipMemcpyAsync(hw.data(), work, N * sizeof(double*), hipMemcpyDeviceToHost, s));
    DD_HIP(hipStreamSynchronize(s));
    int nmax = 0;
    for (int b = 0; b < N; ++b) {
        const int n = H.h[b].n;
        nmax = std::max(nmax, n);
        double* base = hw[b];  // n*(K+1) V, n w, 2(K+1) al/be, theta
        double* V = base;
        double* w = V + (int64_t)n * (K + 1);
        double* al = w + n;
        double* be = al + (K + 1);
        double* th = be + (K + 1);
        lz.h.push_back(LzItem{H.h[b], V, w, al, be, dsteps + b, dout + b});
    }
    lz.sync(s);
    DBuf<double> hbuf((int64_t)std::max(1, N) * 2 * (K + 1));
    std::vector<double*> hh(N);
    for (int b = 0; b < N; ++b) hh[b] = hbuf.p + (int64_t)b * 2 * (K + 1);
    DBuf<double*> hp(std::max(1, N));
    h2d(hp.p, hh.data(), N, s);
    hipLaunchKernelGGL(k_lz_init, dim3(N), dim3(256), 0, s, lz.d.p, N);
    launch_check("lz_init");
    std::vector<int> hdone(N);
    const int Kmax = std::min(K, nmax);
    for (int j = 0; j < Kmax; ++j) {
        int64_t nt = 0, nd = 0, nu = 0, nf = 0;
        for (int b = 0; b < N; ++b)
            if (!hdone[b] && j < H.h[b].n) {
                nt += ceil_div(H.h[b].n, 64);
                nd += (j + 16) / 16;
                nu += ceil_div(H.h[b].n, 256);
                ++nf;
            }
        if (nt == 0) break;
        launch_tiles(OpLzMatvec{lz.d.p, j}, N, nt, s, "lz_matvec");
        for (int pass = 0; pass < 2; ++pass) {
            launch_tiles(OpLzDots{lz.d.p, hp.p, j, K, pass}, N, nd, s, "lz_dots");
            launch_tiles(OpLzUpd{lz.d.p, hp.p, j, K, pass}, N, nu, s, "lz_upd");
        }
        launch_tiles(OpLzFinish{lz.d.p, hp.p, j, K}, N, nf, s, "lz_finish");
        if (j % 8 == 7) {
            DD_HIP(hipMemcpyAsync(hdone.data(), dsteps, N * sizeof(int), hipMemcpyDeviceToHost, s));
            DD_HIP(hipStreamSynchronize(s));
        }
    }
    DD_HIP(hipStreamSynchronize(s));
}

}  // namespace dd
