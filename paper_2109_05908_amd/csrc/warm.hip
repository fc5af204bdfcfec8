// Learned start blocks for the block eigensolver: boundary-node features,
// the network's forward, gradient and Adam kernels, and the sparse products of
// the start block (gfx950, FP64).
#include "warm.hpp"

#include <algorithm>

namespace dd {

__device__ __forceinline__ int bsearch_i32(const int32_t* a, int n, int key) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = a[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}
// largest i in [0, n) with off[i] <= e (off ascending, off[0] = 0)
__device__ __forceinline__ int find_seg(const int64_t* off, int n, int64_t e) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ double diag_of(const CsrDev& A, int r) {
    const int b = A.rowptr[r], e = A.rowptr[r + 1];
    const int k = bsearch_i32(A.colind + b, e - b, r);
    return k >= 0 ? fabs(A.val[b + k]) : 0.0;
}
__device__ __forceinline__ double safe_log(double x) { return log(fmax(x, 1e-300)); }
// local index of global g in Omega_i = [I_i, Gamma_i] (-1 if outside)
__device__ __forceinline__ int omega_index(const int32_t* base, int nI, int nG, int g) {
    const int li = bsearch_i32(base, nI, g);
    if (li >= 0) return li;
    const int lg = bsearch_i32(base + nI, nG, g);
    return lg >= 0 ? nI + lg : -1;
}

// ===========================================================================
// features
// ===========================================================================
__global__ void k_logdiag(WsMaps M, double* smean) {
    __shared__ double red[4];
    const int i = blockIdx.x;
    const int ni = M.counts[3 * i] + M.counts[3 * i + 1];
    const int32_t* base = M.ext + M.offE[i];
    double acc = 0.0;
    for (int r = threadIdx.x; r < ni; r += blockDim.x) acc += safe_log(diag_of(M.A, base[r]));
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) smean[i] = ni ? acc / ni : 0.0;
}
void ws_subdomain_logdiag(const WsMaps& M, double* smean, hipStream_t s) {
    hipLaunchKernelGGL(k_logdiag, dim3(M.N), dim3(256), 0, s, M, smean);
    launch_check("ws_logdiag");
}

// Features of boundary node d of subdomain i (everything relative to the mean
// log diagonal of Omega_i, so they do not change when A is scaled):
//  0 log a_dd;  1 log of the fraction of d's coupling that goes into Omega_i;
//  2 log of d's strongest link into Omega_i;  3 share of d's neighbours in Omega_i;
//  4 log of d's total off-diagonal coupling;  5 mean log diagonal of those neighbours;
//  6 log of the strongest link from those neighbours on into Omega_i (two hops);
//  7 log of the largest diagonal among them.
__global__ void k_features(WsMaps M, const double* smean, const int64_t* offD, int64_t total, double* feats) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = find_seg(offD, M.N, e);
        const int a = (int)(e - offD[i]);
        const int nI = M.counts[3 * i], nG = M.counts[3 * i + 1];
        const int32_t* base = M.ext + M.offE[i];
        const int d = base[nI + nG + a];
        const double sm = smean[i];
        double add = 0.0, in_sum = 0.0, in_max = 0.0, all_sum = 0.0, in_ld = 0.0, hop = 0.0, in_dmax = 0.0;
        int deg = 0, in_cnt = 0;
        for (int q = M.A.rowptr[d]; q < M.A.rowptr[d + 1]; ++q) {
            const int c = M.A.colind[q];
            const double v = fabs(M.A.val[q]);
            if (c == d) {
                add = v;
                continue;
            }
            ++deg;
            all_sum += v;
            if (omega_index(base, nI, nG, c) < 0) continue;
            ++in_cnt;
            in_sum += v;
            in_max = fmax(in_max, v);
            const double ac = diag_of(M.A, c);
            in_ld += safe_log(ac);
            in_dmax = fmax(in_dmax, ac);
            for (int q2 = M.A.rowptr[c]; q2 < M.A.rowptr[c + 1]; ++q2) {
                const int u = M.A.colind[q2];
                if (u != c && omega_index(base, nI, nG, u) >= 0) hop = fmax(hop, fabs(M.A.val[q2]));
            }
        }
        double* f = feats + e * WS_F;
        f[0] = safe_log(add) - sm;
        f[1] = safe_log(in_sum) - safe_log(add);
        f[2] = safe_log(in_max) - sm;
        f[3] = deg ? (double)in_cnt / deg : 0.0;
        f[4] = safe_log(all_sum) - sm;
        f[5] = in_cnt ? in_ld / in_cnt - sm : 0.0;
        f[6] = safe_log(hop) - sm;
        f[7] = safe_log(in_dmax) - sm;
    }
}
void ws_features(const WsMaps& M, const double* smean, const int64_t* offD, int64_t total, double* feats,
                 hipStream_t s) {
    if (total <= 0) return;
    const int g = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_features, dim3(g), dim3(256), 0, s, M, smean, offD, total, feats);
    launch_check("ws_features");
}

// ===========================================================================
// sparse products of the start block and of the training target
// ===========================================================================
constexpr int WS_CHUNK = 8;

__global__ void k_range_product(WsMaps M, const int64_t* offO, int64_t rows, const int64_t* offD, const double* w,
                                double* const* G, double* const* B, const int32_t* kcols) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = find_seg(offO, M.N, e);
        const int r = (int)(e - offO[i]);
        const int nI = M.counts[3 * i], nG = M.counts[3 * i + 1], nD = M.counts[3 * i + 2];
        const int ni = nI + nG, k = kcols[i];
        const int32_t* base = M.ext + M.offE[i];
        const int g = base[r];
        const double* Gi = G[i];
        double* Bi = B[i];
        for (int j0 = 0; j0 < k; j0 += WS_CHUNK) {
            double acc[WS_CHUNK];
#pragma unroll
            for (int j = 0; j < WS_CHUNK; ++j) acc[j] = 0.0;
            for (int q = M.A.rowptr[g]; q < M.A.rowptr[g + 1]; ++q) {
                const int a = bsearch_i32(base + ni, nD, M.A.colind[q]);
                if (a < 0) continue;
                const double coef = M.A.val[q] * (w ? w[offD[i] + a] : 1.0);
#pragma unroll
                for (int j = 0; j < WS_CHUNK; ++j)
                    if (j0 + j < k) acc[j] += coef * Gi[a + (int64_t)(j0 + j) * nD];
            }
#pragma unroll
            for (int j = 0; j < WS_CHUNK; ++j)
                if (j0 + j < k) Bi[r + (int64_t)(j0 + j) * ni] = acc[j];
        }
    }
}
void ws_range_product(const WsMaps& M, const int64_t* offO, int64_t rows, const int64_t* offD, const double* w,
                      double* const* G, double* const* B, const int32_t* kcols, hipStream_t s) {
    if (rows <= 0) return;
    const int g = (int)std::min<int64_t>((rows + 255) / 256, 4096);
    hipLaunchKernelGGL(k_range_product, dim3(g), dim3(256), 0, s, M, offO, rows, offD, w, G, B, kcols);
    launch_check("ws_range_product");
}

__global__ void k_adjoint_product(WsMaps M, const int64_t* offD, int64_t total, double* const* U, double* const* Gt,
                                  const int32_t* pcols) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = find_seg(offD, M.N, e);
        const int a = (int)(e - offD[i]);
        const int nI = M.counts[3 * i], nG = M.counts[3 * i + 1], nD = M.counts[3 * i + 2];
        const int ni = nI + nG, p = pcols[i];
        const int32_t* base = M.ext + M.offE[i];
        const int d = base[ni + a];
        const double* Ui = U[i];
        double* Gi = Gt[i];
        for (int j0 = 0; j0 < p; j0 += WS_CHUNK) {
            double acc[WS_CHUNK];
#pragma unroll
            for (int j = 0; j < WS_CHUNK; ++j) acc[j] = 0.0;
            for (int q = M.A.rowptr[d]; q < M.A.rowptr[d + 1]; ++q) {
                const int lr = omega_index(base, nI, nG, M.A.colind[q]);
                if (lr < 0) continue;
                const double coef = M.A.val[q];
#pragma unroll
                for (int j = 0; j < WS_CHUNK; ++j)
                    if (j0 + j < p) acc[j] += coef * Ui[lr + (int64_t)(j0 + j) * ni];
            }
#pragma unroll
            for (int j = 0; j < WS_CHUNK; ++j)
                if (j0 + j < p) Gi[a + (int64_t)(j0 + j) * nD] = acc[j];
        }
    }
}
void ws_adjoint_product(const WsMaps& M, const int64_t* offD, int64_t total, double* const* U, double* const* Gt,
                        const int32_t* pcols, hipStream_t s) {
    if (total <= 0) return;
    const int g = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_adjoint_product, dim3(g), dim3(256), 0, s, M, offD, total, U, Gt, pcols);
    launch_check("ws_adjoint_product");
}

__global__ void k_row_leverage(const RowItem* items) {
    const RowItem it = items[blockIdx.y];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < it.m; r += gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int j = 0; j < it.n; ++j) {
            const double v = it.Q[r + (int64_t)j * it.ld];
            a += v * v;
        }
        it.out[r] = a * it.scale;
    }
}
void ws_row_leverage(Batch<RowItem>& b, hipStream_t s) {
    if (!b.size()) return;
    hipLaunchKernelGGL(k_row_leverage, dim3(16, b.size()), dim3(256), 0, s, b.d.p);
    launch_check("ws_row_leverage");
}

// ===========================================================================
// the network
// ===========================================================================
// parameter offsets
constexpr int P_W1 = 0;
constexpr int P_B1 = P_W1 + WS_H * WS_F;
constexpr int P_W2 = P_B1 + WS_H;
constexpr int P_B2 = P_W2 + WS_H * WS_H;
constexpr int P_W3 = P_B2 + WS_H;
constexpr int P_B3 = P_W3 + WS_H;
static_assert(P_B3 + 1 == WS_P, "parameter layout");

__device__ __forceinline__ double softplus(double o) { return o > 0.0 ? o + log1p(exp(-o)) : log1p(exp(o)); }
__device__ __forceinline__ double sigmoid(double o) {
    return o >= 0.0 ? 1.0 / (1.0 + exp(-o)) : exp(o) / (1.0 + exp(o));
}

// one sample's forward pass; x (standardised input), h1, h2 (hidden), returns o
__device__ __forceinline__ double mlp_fwd1(const double* P, const double* x, double* h1, double* h2) {
    for (int h = 0; h < WS_H; ++h) {
        double z = P[P_B1 + h];
        for (int f = 0; f < WS_F; ++f) z += P[P_W1 + h * WS_F + f] * x[f];
        h1[h] = tanh(z);
    }
    for (int h = 0; h < WS_H; ++h) {
        double z = P[P_B2 + h];
        for (int g = 0; g < WS_H; ++g) z += P[P_W2 + h * WS_H + g] * h1[g];
        h2[h] = tanh(z);
    }
    double o = P[P_B3];
    for (int h = 0; h < WS_H; ++h) o += P[P_W3 + h] * h2[h];
    return o;
}

__global__ void __launch_bounds__(256) k_mlp_forward(const double* params, const double* mean, const double* stdv,
                                                     const double* feats, int64_t n, double* out) {
    __shared__ double P[WS_P];
    __shared__ double mu[WS_F], sd[WS_F];
    for (int p = threadIdx.x; p < WS_P; p += blockDim.x) P[p] = params[p];
    if (threadIdx.x < WS_F) {
        mu[threadIdx.x] = mean[threadIdx.x];
        sd[threadIdx.x] = stdv[threadIdx.x];
    }
    __syncthreads();
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double x[WS_F], h1[WS_H], h2[WS_H];
        for (int f = 0; f < WS_F; ++f) x[f] = (feats[e * WS_F + f] - mu[f]) / sd[f];
        out[e] = softplus(mlp_fwd1(P, x, h1, h2));
    }
}
void mlp_forward(const double* params, const double* mean, const double* stdv, const double* feats, int64_t n,
                 double* out, hipStream_t s) {
    if (n <= 0) return;
    const int g = (int)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(256), 0, s, params, mean, stdv, feats, n, out);
    launch_check("mlp_forward");
}

// Gradient: each workgroup takes chunks of MLP_CH samples; one thread per sample
// runs the forward and backward pass into LDS, then every thread sums the
// parameter gradients of its parameters over the chunk (fixed order), and the
// workgroup's partial sums go to part[blockIdx.x][p].  A second kernel adds
// the partials in block order: deterministic.
constexpr int MLP_CH = 64;
constexpr int MLP_BLOCKS = 512;
constexpr int MLP_PPT = (WS_P + 255) / 256;  // parameters per thread

__global__ void __launch_bounds__(256) k_mlp_grad(const double* params, const double* mean, const double* stdv,
                                                  const double* feats, const double* target, const double* weight,
                                                  int64_t n, double* part, double* lpart) {
    __shared__ double P[WS_P];
    __shared__ double mu[WS_F], sd[WS_F];
    __shared__ double X[MLP_CH][WS_F], H1[MLP_CH][WS_H], D1[MLP_CH][WS_H], H2[MLP_CH][WS_H], D2[MLP_CH][WS_H];
    __shared__ double DO[MLP_CH];
    __shared__ double red[4];
    for (int p = threadIdx.x; p < WS_P; p += blockDim.x) P[p] = params[p];
    if (threadIdx.x < WS_F) {
        mu[threadIdx.x] = mean[threadIdx.x];
        sd[threadIdx.x] = stdv[threadIdx.x];
    }
    double acc[MLP_PPT];
#pragma unroll
    for (int q = 0; q < MLP_PPT; ++q) acc[q] = 0.0;
    double lacc = 0.0;
    __syncthreads();
    for (int64_t c0 = (int64_t)blockIdx.x * MLP_CH; c0 < n; c0 += (int64_t)gridDim.x * MLP_CH) {
        const int t = threadIdx.x;
        if (t < MLP_CH) {
            const int64_t e = c0 + t;
            if (e < n) {
                double x[WS_F], h1[WS_H], h2[WS_H];
                for (int f = 0; f < WS_F; ++f) x[f] = (feats[e * WS_F + f] - mu[f]) / sd[f];
                const double o = mlp_fwd1(P, x, h1, h2);
                const double wv = softplus(o);
                const double diff = wv - target[e];
                lacc += weight[e] * diff * diff;
                const double dout = 2.0 * weight[e] * diff * sigmoid(o);  // dL/do
                DO[t] = dout;
                for (int f = 0; f < WS_F; ++f) X[t][f] = x[f];
                for (int h = 0; h < WS_H; ++h) {
                    H1[t][h] = h1[h];
                    H2[t][h] = h2[h];
                    D2[t][h] = dout * P[P_W3 + h] * (1.0 - h2[h] * h2[h]);  // dL/dz2
                }
                for (int g = 0; g < WS_H; ++g) {
                    double a = 0.0;
                    for (int h = 0; h < WS_H; ++h) a += P[P_W2 + h * WS_H + g] * D2[t][h];
                    D1[t][g] = a * (1.0 - h1[g] * h1[g]);  // dL/dz1
                }
            } else {
                DO[t] = 0.0;
                for (int f = 0; f < WS_F; ++f) X[t][f] = 0.0;
                for (int h = 0; h < WS_H; ++h) {
                    H1[t][h] = 0.0;
                    H2[t][h] = 0.0;
                    D1[t][h] = 0.0;
                    D2[t][h] = 0.0;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MLP_PPT; ++q) {
            const int p = threadIdx.x + q * 256;
            if (p >= WS_P) continue;
            double a = 0.0;
            if (p < P_B1) {
                const int h = (p - P_W1) / WS_F, f = (p - P_W1) % WS_F;
                for (int c = 0; c < MLP_CH; ++c) a += D1[c][h] * X[c][f];
            } else if (p < P_W2) {
                const int h = p - P_B1;
                for (int c = 0; c < MLP_CH; ++c) a += D1[c][h];
            } else if (p < P_B2) {
                const int h = (p - P_W2) / WS_H, g = (p - P_W2) % WS_H;
                for (int c = 0; c < MLP_CH; ++c) a += D2[c][h] * H1[c][g];
            } else if (p < P_W3) {
                const int h = p - P_B2;
                for (int c = 0; c < MLP_CH; ++c) a += D2[c][h];
            } else if (p < P_B3) {
                const int h = p - P_W3;
                for (int c = 0; c < MLP_CH; ++c) a += DO[c] * H2[c][h];
            } else {
                for (int c = 0; c < MLP_CH; ++c) a += DO[c];
            }
            acc[q] += a;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < MLP_PPT; ++q) {
        const int p = threadIdx.x + q * 256;
        if (p < WS_P) part[(int64_t)blockIdx.x * WS_P + p] = acc[q];
    }
    lacc = block_sum(lacc, red);
    if (threadIdx.x == 0) lpart[blockIdx.x] = lacc;
}

__global__ void k_mlp_reduce(const double* part, const double* lpart, int nb, double* grad, double* loss) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= WS_P; p += gridDim.x * blockDim.x) {
        double a = 0.0;
        if (p < WS_P) {
            for (int b = 0; b < nb; ++b) a += part[(int64_t)b * WS_P + p];
            grad[p] = a;
        } else {
            for (int b = 0; b < nb; ++b) a += lpart[b];
            *loss = a;
        }
    }
}

void mlp_loss_grad(const double* params, const double* mean, const double* stdv, const double* feats,
                   const double* target, const double* weight, int64_t n, double* grad, double* dloss,
                   hipStream_t s) {
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + MLP_CH - 1) / MLP_CH, MLP_BLOCKS));
    DBuf<double> part((size_t)nb * WS_P), lpart(nb);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, params, mean, stdv, feats, target, weight, n, part.p,
                       lpart.p);
    launch_check("mlp_grad");
    hipLaunchKernelGGL(k_mlp_reduce, dim3((WS_P + 256) / 256), dim3(256), 0, s, part.p, lpart.p, nb, grad, dloss);
    launch_check("mlp_reduce");
    DD_HIP(hipStreamSynchronize(s));  // part, lpart are freed on return
}

__global__ void k_adam(double* params, const double* grad, double* m1, double* m2, double lr, double c1, double c2) {
    constexpr double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < WS_P; p += gridDim.x * blockDim.x) {
        const double g = grad[p];
        const double m = b1 * m1[p] + (1.0 - b1) * g;
        const double v = b2 * m2[p] + (1.0 - b2) * g * g;
        m1[p] = m;
        m2[p] = v;
        params[p] -= lr * (m / c1) / (sqrt(v / c2) + eps);
    }
}
void mlp_adam(double* params, const double* grad, double* m1, double* m2, double lr, int t, hipStream_t s) {
    const double c1 = 1.0 - std::pow(0.9, t), c2 = 1.0 - std::pow(0.999, t);
    hipLaunchKernelGGL(k_adam, dim3((WS_P + 255) / 256), dim3(256), 0, s, params, grad, m1, m2, lr, c1, c2);
    launch_check("mlp_adam");
}

__global__ void k_feature_stats(const double* feats, int64_t n, double* mean, double* stdv) {
    __shared__ double red[4];
    const int f = blockIdx.x;
    double a = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) a += feats[e * WS_F + f];
    a = block_sum(a, red);
    const double m = n ? a / n : 0.0;
    double v = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
        const double d = feats[e * WS_F + f] - m;
        v += d * d;
    }
    v = block_sum(v, red);
    if (threadIdx.x == 0) {
        mean[f] = m;
        const double sd = n > 1 ? sqrt(v / (n - 1)) : 1.0;
        stdv[f] = sd > 1e-12 ? sd : 1.0;
    }
}
void ws_feature_stats(const double* feats, int64_t n, double* mean, double* stdv, hipStream_t s) {
    hipLaunchKernelGGL(k_feature_stats, dim3(WS_F), dim3(256), 0, s, feats, n, mean, stdv);
    launch_check("ws_feature_stats");
}

}  // namespace dd
