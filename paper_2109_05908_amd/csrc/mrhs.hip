// Multi-column local solves: the triangular matrix-vector products of
// dense.hip (OpTrmvN, OpTrmvRed, OpTrmvT, OpTrmvTRed) with the same tiles and
// summation order per column, each loaded entry of W used for every column.
#include "mrhs.hpp"

namespace dd {

template <class TW>
struct OpTrmvNM {
    const TrmvMItem<TW>* it;
    int nrhs;
    __device__ static int nrb(int n) { return (n + TRMV_RB - 1) / TRMV_RB; }
    __device__ static int ncc(int n) { return (n + TRMV_CC - 1) / TRMV_CC; }
    __device__ int tiles(int b) const { return nrb(it[b].n) * ncc(it[b].n); }
    __device__ void operator()(int b, int t) const {
        __shared__ double red[kMrhs][4][TRMV_RB];
        const TrmvMItem<TW>& I = it[b];
        const int n = I.n, nc = ncc(n), kn = nrhs;
        const int rb = t / nc, cc = t % nc;
        const int r0 = rb * TRMV_RB, c0 = cc * TRMV_CC;
        if (c0 > r0 + TRMV_RB - 1) return;  // above the diagonal: no partial
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int r = r0 + lane;
        const int cend = min(min(c0 + TRMV_CC, n), r0 + TRMV_RB);
        TW a[kMrhs][4];
#pragma unroll
        for (int k = 0; k < kMrhs; ++k) a[k][0] = a[k][1] = a[k][2] = a[k][3] = 0;
        if (r < n) {
            const TW* Wr = I.W + r;
            int j = c0 + w;
            for (; j + 12 < cend; j += 16) {
                const TW w0 = Wr[(int64_t)j * I.ld], w1 = Wr[(int64_t)(j + 4) * I.ld];
                const TW w2 = Wr[(int64_t)(j + 8) * I.ld], w3 = Wr[(int64_t)(j + 12) * I.ld];
#pragma unroll
                for (int k = 0; k < kMrhs; ++k) {
                    if (k < kn) {
                        const double* xk = I.x + (int64_t)k * I.xs;
                        a[k][0] += w0 * (TW)xk[j];
                        a[k][1] += w1 * (TW)xk[j + 4];
                        a[k][2] += w2 * (TW)xk[j + 8];
                        a[k][3] += w3 * (TW)xk[j + 12];
                    }
                }
            }
            for (; j < cend; j += 4) {
                const TW w0 = Wr[(int64_t)j * I.ld];
#pragma unroll
                for (int k = 0; k < kMrhs; ++k)
                    if (k < kn) a[k][0] += w0 * (TW)I.x[(int64_t)k * I.xs + j];
            }
        }
#pragma unroll
        for (int k = 0; k < kMrhs; ++k)
            if (k < kn) red[k][w][lane] = (double)((a[k][0] + a[k][1]) + (a[k][2] + a[k][3]));
        __syncthreads();
        if (w == 0 && r < n)
            for (int k = 0; k < kn; ++k)
                I.part[(int64_t)k * I.ps + (int64_t)cc * n + r] =
                    (red[k][0][lane] + red[k][1][lane]) + (red[k][2][lane] + red[k][3][lane]);
    }
};

template <class TW>
struct OpTrmvRedM {
    const TrmvMItem<TW>* it;
    int nrhs;
    __device__ int tiles(int b) const { return (it[b].n + 255) / 256; }
    __device__ void operator()(int b, int t) const {
        const TrmvMItem<TW>& I = it[b];
        const int r = t * 256 + threadIdx.x;
        if (r >= I.n) return;
        const int last = ((r / TRMV_RB) * TRMV_RB + TRMV_RB - 1) / TRMV_CC;
        for (int k = 0; k < nrhs; ++k) {
            const double* pk = I.part + (int64_t)k * I.ps;
            double v = 0.0;
            for (int cc = 0; cc <= last; ++cc) v += pk[(int64_t)cc * I.n + r];
            I.y[(int64_t)k * I.ys + r] = v;
        }
    }
};

template <class TW>
struct OpTrmvTM {
    const TrmvMItem<TW>* it;
    int nrhs;
    __device__ int tiles(int b) const { return trmv_t_tiles(it[b].n); }
    __device__ void operator()(int b, int t) const {
        const TrmvMItem<TW>& I = it[b];
        const int n = I.n, kn = nrhs;
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
        TW accw[kMrhs][4];
#pragma unroll
        for (int k = 0; k < kMrhs; ++k) accw[k][0] = accw[k][1] = accw[k][2] = accw[k][3] = 0;
        if (j0 < n) {
            const int jn = min(4, n - j0);
            for (int i = rb + lane; i < re; i += 64) {
                TW wq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) wq[q] = (q < jn) ? I.W[i + (int64_t)(j0 + q) * I.ld] : TW(0);
#pragma unroll
                for (int k = 0; k < kMrhs; ++k) {
                    if (k < kn) {
                        const TW yi = (TW)I.y[(int64_t)k * I.ys + i];
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (q < jn) accw[k][q] += wq[q] * yi;
                    }
                }
            }
        }
        for (int k = 0; k < kn; ++k) {
            double acc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = wave_sum((double)accw[k][q]);
            if (lane == 0)
                for (int q = 0; q < 4; ++q)
                    if (j0 + q < n) I.part[(int64_t)k * I.ps + (int64_t)c * n + j0 + q] = acc[q];
        }
    }
};

template <class TW>
struct OpTrmvTRedM {
    const TrmvMItem<TW>* it;
    int nrhs;
    __device__ int tiles(int b) const { return (it[b].n + 255) / 256; }
    __device__ void operator()(int b, int t) const {
        const TrmvMItem<TW>& I = it[b];
        const int j = t * 256 + threadIdx.x;
        if (j >= I.n) return;
        const int nch = (I.n + TRMV_CC - 1) / TRMV_CC;
        for (int k = 0; k < nrhs; ++k) {
            const double* pk = I.part + (int64_t)k * I.ps;
            double v = 0.0;
            for (int c = j / TRMV_CC; c < nch; ++c) v += pk[(int64_t)c * I.n + j];
            I.x[(int64_t)k * I.xs + j] = v;
        }
    }
};

template <class TW>
static void trinv_multi(Batch<TrmvMItem<TW>>& t, int nrhs, hipStream_t s) {
    DD_CHECK(nrhs >= 1 && nrhs <= kMrhs, DD_ERR_INTERNAL, "multi-column local solve: 1..8 columns");
    int64_t tn = 0, tt = 0, tr = 0;
    for (auto& x : t.h) {
        tn += (int64_t)ceil_div(x.n, TRMV_RB) * ceil_div(x.n, TRMV_CC);
        tt += trmv_t_tiles(x.n);
        tr += ceil_div(x.n, 256);
    }
    launch_tiles(OpTrmvNM<TW>{t.d.p, nrhs}, t.size(), tn, s, "trmv_n_multi");
    launch_tiles(OpTrmvRedM<TW>{t.d.p, nrhs}, t.size(), tr, s, "trmv_red_multi");
    launch_tiles(OpTrmvTM<TW>{t.d.p, nrhs}, t.size(), tt, s, "trmv_t_multi");
    launch_tiles(OpTrmvTRedM<TW>{t.d.p, nrhs}, t.size(), tr, s, "trmv_t_red_multi");
}

void trinv_apply_multi_vb(Batch<TrmvMItem<double>>& t, int nrhs, hipStream_t s) { trinv_multi(t, nrhs, s); }
void trinv_apply_multi_vb(Batch<TrmvMItem<float>>& t, int nrhs, hipStream_t s) { trinv_multi(t, nrhs, s); }

}  // namespace dd
