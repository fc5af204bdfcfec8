// LOBPCG for the local eigenproblem (3.3) in cap mode, and the batched Jacobi
// eigensolver of its Rayleigh-Ritz steps (gfx950).
#include "lobpcg.hpp"

#include <algorithm>
#include <cmath>

namespace dd {

// ===========================================================================
// Jacobi
// ===========================================================================
constexpr int JAC_LD = JAC_MAX + 1;
constexpr int JAC_THREADS = 1024;  // one workgroup per CU either way (its LDS): more threads shorten every round

// Round r of the circle method on mp (even) players: pair 0 is (r, mp - 1),
// pair j >= 1 is ((r + j) mod (mp - 1), (r - j) mod (mp - 1)); every pair of
// players meets once in mp - 1 rounds.
__device__ __forceinline__ void rr_pair(int r, int j, int mp, int& p, int& q) {
    const int m1 = mp - 1;
    if (j == 0) {
        p = r;
        q = m1;
    } else {
        p = (r + j) % m1;
        q = (r - j + m1) % m1;
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

__global__ void __launch_bounds__(JAC_THREADS) k_jacobi(const JacItem* items, int max_sweeps) {
    __shared__ double A[JAC_MAX * JAC_LD];
    __shared__ double cs[JAC_MAX / 2], sn[JAC_MAX / 2];
    __shared__ int pp[JAC_MAX / 2], qq[JAC_MAX / 2];
    __shared__ double red[JAC_THREADS / 64];
    __shared__ int order[JAC_MAX];
    __shared__ double wv[JAC_MAX];
    const JacItem it = items[blockIdx.x];
    const int m = it.m;
    if (m <= 0) return;
    const int mp = m + (m & 1);
    const int t = threadIdx.x;
    // load (A + A^T) / 2, zero padding; V := I (columns in global memory)
    for (int e = t; e < mp * mp; e += blockDim.x) {
        const int r = e % mp, c = e / mp;
        double v = 0.0;
        if (r < m && c < m) v = 0.5 * (it.A[r + (int64_t)c * it.lda] + it.A[c + (int64_t)r * it.lda]);
        A[r + c * JAC_LD] = v;
    }
    for (int e = t; e < m * m; e += blockDim.x) {
        const int r = e % m, c = e / m;
        it.V[r + (int64_t)c * it.ldv] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    double fro2 = 0.0;
    for (int e = t; e < mp * mp; e += blockDim.x) {
        const double v = A[(e % mp) + (e / mp) * JAC_LD];
        fro2 += v * v;
    }
    fro2 = block_sum(fro2, red);
    const int npair = mp / 2;
    for (int sweep = 0; sweep < max_sweeps && mp > 1; ++sweep) {
        double off = 0.0;
        for (int e = t; e < mp * mp; e += blockDim.x) {
            const int r = e % mp, c = e / mp;
            if (r != c) {
                const double v = A[r + c * JAC_LD];
                off += v * v;
            }
        }
        off = block_sum(off, red);
        if (!(off > 1e-30 * fro2)) break;  // off-diagonal below (1e-15 ||A||_F)^2
        for (int r = 0; r < mp - 1; ++r) {
            // rotation angles (Golub & Van Loan, symmetric Schur 2x2)
            for (int j = t; j < npair; j += blockDim.x) {
                int p, q;
                rr_pair(r, j, mp, p, q);
                pp[j] = p;
                qq[j] = q;
                const double apq = A[p + q * JAC_LD];
                double c = 1.0, s = 0.0;
                if (q < m && apq != 0.0) {
                    const double app = A[p + p * JAC_LD], aqq = A[q + q * JAC_LD];
                    const double th = (aqq - app) / (2.0 * apq);
                    const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    c = 1.0 / sqrt(tt * tt + 1.0);
                    s = tt * c;
                }
                cs[j] = c;
                sn[j] = s;
            }
            __syncthreads();
            // rows: A := J^T A
            for (int e = t; e < npair * mp; e += blockDim.x) {
                const int j = e / mp, l = e % mp;
                const double c = cs[j], s = sn[j];
                if (s == 0.0) continue;
                const int p = pp[j], q = qq[j];
                const double ap = A[p + l * JAC_LD], aq = A[q + l * JAC_LD];
                A[p + l * JAC_LD] = c * ap - s * aq;
                A[q + l * JAC_LD] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A := A J, and V := V J
            for (int e = t; e < npair * mp; e += blockDim.x) {
                const int j = e / mp, l = e % mp;
                const double c = cs[j], s = sn[j];
                if (s == 0.0) continue;
                const int p = pp[j], q = qq[j];
                const double ap = A[l + p * JAC_LD], aq = A[l + q * JAC_LD];
                A[l + p * JAC_LD] = c * ap - s * aq;
                A[l + q * JAC_LD] = s * ap + c * aq;
                if (l < m) {
                    double* vp = it.V + (int64_t)p * it.ldv;
                    double* vq = it.V + (int64_t)q * it.ldv;
                    const double xp = vp[l], xq = vq[l];
                    vp[l] = c * xp - s * xq;
                    vq[l] = s * xp + c * xq;
                }
            }
            __syncthreads();
            for (int j = t; j < npair; j += blockDim.x)
                if (sn[j] != 0.0) {  // annihilated exactly
                    A[pp[j] + qq[j] * JAC_LD] = 0.0;
                    A[qq[j] + pp[j] * JAC_LD] = 0.0;
                }
            __syncthreads();
        }
    }
    // eigenvalues descending (rank by comparison, ties by index; a NaN ranks
    // as -inf, so the ranks always form a permutation), then reorder V
    for (int i = t; i < m; i += blockDim.x) {
        const double v = A[i + i * JAC_LD];
        wv[i] = (v == v) ? v : -INFINITY;
    }
    __syncthreads();
    for (int i = t; i < m; i += blockDim.x) {
        const double v = wv[i];
        int rank = 0;
        for (int j = 0; j < m; ++j) rank += (wv[j] > v || (wv[j] == v && j < i)) ? 1 : 0;
        order[rank] = i;
        it.w[rank] = A[i + i * JAC_LD];
    }
    __syncthreads();
    // permute the columns of V through LDS (A's storage is free now)
    for (int e = t; e < m * m; e += blockDim.x) {
        const int r = e % m, c = e / m;
        A[r + c * JAC_LD] = it.V[r + (int64_t)order[c] * it.ldv];
    }
    __syncthreads();
    for (int e = t; e < m * m; e += blockDim.x) {
        const int r = e % m, c = e / m;
        it.V[r + (int64_t)c * it.ldv] = A[r + c * JAC_LD];
    }
}

void jacobi_eig_vb(Batch<JacItem>& b, hipStream_t s) {
    if (!b.size()) return;
    for (const auto& it : b.h) DD_CHECK(it.m <= JAC_MAX, DD_ERR_INTERNAL, "Jacobi: matrix larger than JAC_MAX");
    hipLaunchKernelGGL(k_jacobi, dim3(b.size()), dim3(JAC_THREADS), 0, s, b.d.p, 40);
    launch_check("jacobi");
}

// ===========================================================================
// small kernels
// ===========================================================================
__device__ __forceinline__ uint64_t smix(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// standard normal from two counter draws (Box-Muller, cosine branch)
__device__ __forceinline__ double gauss_at(uint64_t seed, uint64_t k) {
    const double u1 = ((smix(seed, 2 * k) >> 11) + 1.0) * 0x1.0p-53;   // (0, 1]
    const double u2 = (smix(seed, 2 * k + 1) >> 11) * 0x1.0p-53;       // [0, 1)
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__global__ void k_gaussian(const RandItem* items) {
    const RandItem it = items[blockIdx.y];
    const int64_t tot = (int64_t)it.m * it.n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % it.m), c = (int)(e / it.m);
        it.X[r + (int64_t)c * it.ld] = gauss_at(it.seed, (uint64_t)e);
    }
}
void gaussian_vb(Batch<RandItem>& b, hipStream_t s) {
    if (!b.size()) return;
    hipLaunchKernelGGL(k_gaussian, dim3(64, b.size()), dim3(256), 0, s, b.d.p);
    launch_check("gaussian");
}

__global__ void k_colnorm2(const ColItem* items) {
    __shared__ double red[4];
    const ColItem it = items[blockIdx.y];
    const int j = blockIdx.x;
    if (j >= it.n) return;
    const double* y = it.Y + (int64_t)j * it.ld;
    double a = 0.0;
    for (int r = threadIdx.x; r < it.m; r += blockDim.x) a += y[r] * y[r];
    a = block_sum(a, red);
    if (threadIdx.x == 0) it.out[j] = a;
}
// X[:, j] := X[:, j] / ||X[:, j]|| + eps G[:, j] / ||G[:, j]|| (a zero column of X
// becomes G's): a structured block stays full rank
__global__ void k_mix(const MixItem* items) {
    __shared__ double red[4];
    const MixItem it = items[blockIdx.y];
    const int j = blockIdx.x;
    if (j >= it.k) return;
    double* x = it.X + (int64_t)j * it.n;
    const double* g = it.G + (int64_t)j * it.n;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < it.n; i += blockDim.x) {
        a += x[i] * x[i];
        b += g[i] * g[i];
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    const double sx = a > 0.0 ? 1.0 / sqrt(a) : 0.0, sg = b > 0.0 ? (a > 0.0 ? it.eps : 1.0) / sqrt(b) : 0.0;
    for (int i = threadIdx.x; i < it.n; i += blockDim.x) x[i] = x[i] * sx + g[i] * sg;
}
void colnorm2_vb(Batch<ColItem>& b, hipStream_t s) {
    if (!b.size()) return;
    int nmax = 1;
    for (const auto& it : b.h) nmax = std::max(nmax, it.n);
    hipLaunchKernelGGL(k_colnorm2, dim3(nmax, b.size()), dim3(256), 0, s, b.d.p);
    launch_check("colnorm2");
}

void mix_random_vb(Batch<MixItem>& b, hipStream_t s) {
    if (!b.size()) return;
    int kmax = 1;
    for (const auto& it : b.h) kmax = std::max(kmax, it.k);
    hipLaunchKernelGGL(k_mix, dim3(kmax, b.size()), dim3(256), 0, s, b.d.p);
    launch_check("mix_random");
}

// R = KX - X diag(theta) into R and rho[j] = ||r_j|| / |theta_j| (relative:
// the largest-eigenvalue form) or ||r_j|| (absolute: the smallest-eigenvalue
// form, whose operator has norm <= 1).  Soft locking: a pair whose residual is
// at the stopping level (with the rounding floor of the relative form) has its
// residual and its P direction zeroed, so that no noise-level direction enters
// the next basis (where normalisation would blow it up).
struct ResItem {
    const double* X;
    const double* KX;
    double* R;
    double* P;    // n x k, may be null (no P yet)
    int n, k;
    const double* theta;
    double* rho;
};
__global__ void k_residual(const ResItem* items, int relative, double tol) {
    __shared__ double red[4];
    const ResItem it = items[blockIdx.y];
    const int j = blockIdx.x;
    if (j >= it.k) return;
    const double th = it.theta[j];
    const double* x = it.X + (int64_t)j * it.n;
    const double* kx = it.KX + (int64_t)j * it.n;
    double* r = it.R + (int64_t)j * it.n;
    double a = 0.0;
    for (int i = threadIdx.x; i < it.n; i += blockDim.x) {
        const double v = kx[i] - th * x[i];
        r[i] = v;
        a += v * v;
    }
    a = block_sum(a, red);
    double rho;
    bool lock;
    if (th == 0.0) {  // a zero column (dropped direction) is never converged
        rho = INFINITY;
        lock = false;
    } else if (relative) {
        rho = sqrt(a) / fabs(th);
        const double floor = (th > 0.0) ? 64.0 * 2.220446049250313e-16 * it.theta[0] / th : 0.0;
        lock = rho <= tol + floor;
    } else {
        rho = sqrt(a);
        lock = rho <= tol;
    }
    if (threadIdx.x == 0) it.rho[j] = rho;
    if (lock) {
        for (int i = threadIdx.x; i < it.n; i += blockDim.x) {
            r[i] = 0.0;
            if (it.P) it.P[i + (int64_t)j * it.n] = 0.0;
        }
    }
}
// Smallest-eigenvalue form: a column of the basis W that SVQB dropped (exactly
// zero) would give a Ritz value 0 that beats every wanted one; its diagonal in
// the negated Rayleigh-Ritz matrix is set below every true Ritz value, so it is
// never selected.
struct ZeroColItem {
    const double* W;
    int n, m;
    double* H;  // m x m
};
__global__ void k_exclude_zero_cols(const ZeroColItem* items) {
    __shared__ int nz;
    const ZeroColItem it = items[blockIdx.y];
    const int j = blockIdx.x;
    if (j >= it.m) return;
    if (threadIdx.x == 0) nz = 0;
    __syncthreads();
    const double* w = it.W + (int64_t)j * it.n;
    for (int i = threadIdx.x; i < it.n; i += blockDim.x)
        if (w[i] != 0.0) nz = 1;
    __syncthreads();
    // the Ritz values of S~ lie in [0, 1] (its eigenvalues mu <= 1), those of -H in [-1, 0]
    if (threadIdx.x == 0 && !nz) it.H[j + (int64_t)j * it.m] = -4.0;
}
__global__ void k_negate(const double* src, double* dst, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = -src[i];
}

// SVQB (Stathopoulos & Wu 2002) on a Gram matrix G (kv x kv): D = diag(G)^{-1/2};
// prep: G := D G D; finish (after Jacobi gives U, lambda): T = D U Lambda^{-1/2},
// columns with lambda <= drop * lambda_max set to zero (dependent directions).
struct SvqbItem {
    double* G;
    int kv;
    double* d;   // kv
    const double* U;
    const double* lam;
    double* T;
};
__global__ void k_svqb_prep(const SvqbItem* items) {
    const SvqbItem it = items[blockIdx.x];
    const int kv = it.kv;
    for (int i = threadIdx.x; i < kv; i += blockDim.x) {
        const double g = it.G[i + (int64_t)i * kv];
        it.d[i] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kv * kv; e += blockDim.x) {
        const int r = e % kv, c = e / kv;
        it.G[e] *= it.d[r] * it.d[c];
    }
}
__global__ void k_svqb_finish(const SvqbItem* items, double drop) {
    const SvqbItem it = items[blockIdx.x];
    const int kv = it.kv;
    const double lmax = it.lam[0];
    for (int e = threadIdx.x; e < kv * kv; e += blockDim.x) {
        const int r = e % kv, c = e / kv;
        const double l = it.lam[c];
        it.T[e] = (l > drop * lmax && l > 0.0) ? it.d[r] * it.U[e] / sqrt(l) : 0.0;
    }
}

void orth_basis_vb(std::vector<OrthItem>& items, hipStream_t s) {
    const int nb = (int)items.size();
    if (!nb) return;
    std::vector<int64_t> off(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        const int64_t kv = items[b].kv;
        DD_CHECK(kv >= 1 && kv <= JAC_MAX, DD_ERR_INTERNAL, "orthonormal basis: bad column count");
        off[b + 1] = off[b] + 3 * kv * kv + 2 * kv + 32;
    }
    DBuf<double> buf(off[nb]);
    Batch<GemmItem> g1, g2;
    Batch<SvqbItem> q;
    Batch<JacItem> jb;
    for (int b = 0; b < nb; ++b) {
        const auto& it = items[b];
        const int kv = it.kv;
        double* G = buf.p + off[b];
        double* U = G + kv * kv;
        double* T = U + kv * kv;
        double* lam = T + kv * kv;
        double* d = lam + kv;
        g1.h.push_back(GemmItem{it.V, it.m, it.V, it.m, G, kv, kv, kv, it.m, 1.0, 0.0});
        q.h.push_back(SvqbItem{G, kv, d, U, lam, T});
        jb.h.push_back(JacItem{G, kv, kv, U, kv, lam});
        g2.h.push_back(GemmItem{it.V, it.m, T, kv, it.Q, it.m, it.m, kv, kv, 1.0, 0.0});
    }
    g1.sync(s);
    q.sync(s);
    jb.sync(s);
    g2.sync(s);
    gemm_vb(g1, true, false, s);
    hipLaunchKernelGGL(k_svqb_prep, dim3(nb), dim3(256), 0, s, q.d.p);
    launch_check("svqb_prep");
    jacobi_eig_vb(jb, s);
    hipLaunchKernelGGL(k_svqb_finish, dim3(nb), dim3(256), 0, s, q.d.p, 1e-13);
    launch_check("svqb_finish");
    gemm_vb(g2, false, false, s);
    DD_HIP(hipStreamSynchronize(s));
}

// ===========================================================================
// LOBPCG driver
// ===========================================================================
namespace {

struct Work {  // per item, inside one arena
    double *W, *KW, *P, *T1, *T2, *H, *Ev, *ev, *C1, *G, *Gd, *Tq, *rho, *dv, *Xb, *thb;
};

template <class F>
Batch<GemmItem> gemms(const std::vector<int>& act, F f, hipStream_t s) {
    Batch<GemmItem> g;
    for (int b : act) g.h.push_back(f(b));
    g.sync(s);
    return g;
}

}  // namespace

void lobpcg_vb(std::vector<LobItem>& items, bool matrix_free, double tol, int maxit, hipStream_t s, LobStats& st) {
    // explicit: largest eigenvalues of K = M^T M; matrix-free: smallest of S~ = K^{-1}
    // (operator through L and RL, stable), preconditioned by K applied through the
    // triangular factors (its rounding only slows the iteration, it cannot bias it)
    const bool smallest = matrix_free;
    const int nb = (int)items.size();
    st.iters.assign(nb, 0);
    st.resid.assign(nb, 0.0);
    st.maxit_hits = 0;
    if (!nb) return;
    // workspace
    std::vector<int64_t> off(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        const int64_t n = items[b].n, k = items[b].k, m = 3 * k;
        DD_CHECK(k >= 1 && k <= items[b].n && m <= JAC_MAX, DD_ERR_INTERNAL, "LOBPCG: bad block size");
        const int64_t sz = n * m * 2 + n * k * 2 + n * 2 * k * 2 + m * m * 2 + m + k * 2 * k + 4 * k * k * 3 + 4 * k + n * k;
        off[b + 1] = off[b] + ((sz + 31) / 32) * 32;
    }
    DBuf<double> buf(off[nb]);
    std::vector<Work> w(nb);
    for (int b = 0; b < nb; ++b) {
        const int64_t n = items[b].n, k = items[b].k, m = 3 * k;
        double* p = buf.p + off[b];
        auto take = [&](int64_t c) { double* q = p; p += c; return q; };
        w[b].W = take(n * m);
        w[b].KW = take(n * m);
        w[b].P = take(n * k);
        w[b].T1 = take(n * 2 * k);
        w[b].T2 = take(n * 2 * k);
        w[b].H = take(m * m);
        w[b].Ev = take(m * m);
        w[b].ev = take(m);
        w[b].C1 = take(k * 2 * k);
        w[b].G = take(4 * k * k);
        w[b].Gd = take(4 * k * k);
        w[b].Tq = take(4 * k * k);
        w[b].rho = take(k);
        w[b].dv = take(2 * k);
        w[b].Xb = take(n * k);
        w[b].thb = take(k);
    }
    auto copy_block = [&](const std::vector<int>& act, auto src, auto dst, auto cols) {
        Batch<DMat> a, d;
        for (int b : act) {
            const int n = items[b].n;
            a.h.push_back(DMat{src(b), n, n, cols(b)});
            d.h.push_back(DMat{dst(b), n, n, cols(b)});
        }
        a.sync(s);
        d.sync(s);
        copy_vb(a, d, false, 1.0, s);
    };
    // K applied to the first `cols` columns at in(b) -> out(b); tmp T1 (n x 2k).
    // Explicit: K = M^T M.  Matrix-free: K = L^T RL^{-T} RL^{-1} L (preconditioner).
    auto apply_K = [&](const std::vector<int>& act, auto in, auto out, auto cols) {
        if (!matrix_free) {
            auto g1 = gemms(act, [&](int b) {
                const auto& it = items[b];
                return GemmItem{it.M, it.ldm, in(b), it.n, w[b].T1, it.n, it.n, cols(b), it.n, 1.0, 0.0};
            }, s);
            gemm_vb(g1, false, false, s);
            auto g2 = gemms(act, [&](int b) {
                const auto& it = items[b];
                return GemmItem{it.M, it.ldm, w[b].T1, it.n, out(b), it.n, it.n, cols(b), it.n, 1.0, 0.0};
            }, s);
            gemm_vb(g2, true, false, s);
            return;
        }
        auto g1 = gemms(act, [&](int b) {
            const auto& it = items[b];
            return GemmItem{it.L, it.ldl, in(b), it.n, w[b].T1, it.n, it.n, cols(b), it.n, 1.0, 0.0};
        }, s);
        gemm_vb(g1, false, false, s);
        Batch<DMat> Lr, Bt;
        for (int b : act) {
            Lr.h.push_back(DMat{const_cast<double*>(items[b].RL), items[b].ldr, items[b].n, items[b].n});
            Bt.h.push_back(DMat{w[b].T1, items[b].n, items[b].n, cols(b)});
        }
        Lr.sync(s);
        Bt.sync(s);
        trsm_vb(Lr, Bt, false, s);
        trsm_vb(Lr, Bt, true, s);
        auto g2 = gemms(act, [&](int b) {
            const auto& it = items[b];
            return GemmItem{it.L, it.ldl, w[b].T1, it.n, out(b), it.n, it.n, cols(b), it.n, 1.0, 0.0};
        }, s);
        gemm_vb(g2, true, false, s);
    };
    // the operator whose extreme eigenpairs are wanted: K (explicit) or, matrix-free,
    // S~ = L^{-1} RL RL^T L^{-T} (triangular solves with the well-conditioned L,
    // products with RL): in -> out, temps T1, T2
    auto apply_op = [&](const std::vector<int>& act, auto in, auto out, auto cols) {
        if (!matrix_free) {
            apply_K(act, in, out, cols);
            return;
        }
        Batch<DMat> Lb, Tb, Ib, Ob;
        for (int b : act) {
            Lb.h.push_back(DMat{const_cast<double*>(items[b].L), items[b].ldl, items[b].n, items[b].n});
            Ib.h.push_back(DMat{in(b), items[b].n, items[b].n, cols(b)});
            Tb.h.push_back(DMat{w[b].T1, items[b].n, items[b].n, cols(b)});
            Ob.h.push_back(DMat{out(b), items[b].n, items[b].n, cols(b)});
        }
        Lb.sync(s);
        Tb.sync(s);
        Ib.sync(s);
        Ob.sync(s);
        copy_vb(Ib, Tb, false, 1.0, s);
        trsm_vb(Lb, Tb, true, s);  // T1 = L^{-T} in
        auto g1 = gemms(act, [&](int b) {
            const auto& it = items[b];
            return GemmItem{it.RL, it.ldr, w[b].T1, it.n, w[b].T2, it.n, it.n, cols(b), it.n, 1.0, 0.0};
        }, s);
        gemm_vb(g1, true, false, s);  // T2 = RL^T T1
        auto g2 = gemms(act, [&](int b) {
            const auto& it = items[b];
            return GemmItem{it.RL, it.ldr, w[b].T2, it.n, out(b), it.n, it.n, cols(b), it.n, 1.0, 0.0};
        }, s);
        gemm_vb(g2, false, false, s);  // out = RL T2
        trsm_vb(Lb, Ob, false, s);     // out = L^{-1} out
    };
    auto jacobi = [&](const std::vector<int>& act, auto A, auto m, auto V, auto ev) {
        Batch<JacItem> j;
        for (int b : act) j.h.push_back(JacItem{A(b), m(b), m(b), V(b), m(b), ev(b)});
        j.sync(s);
        jacobi_eig_vb(j, s);
    };
    // SVQB of the first kv(b) columns at Vp(b) (with their K-images at KVp(b) if given)
    // drop: directions with Gram eigenvalue <= drop * largest are removed.  Inside the
    // loop the K-images of P are carried along, and a kept direction of singular value
    // sigma amplifies their rounding by 1 / sigma (with ||K|| ~ 1e14 that creates
    // spurious Ritz values), so there sigma >= 1e-4 is required; the start block's
    // images are computed afresh, so there nearly every direction may stay.
    auto svqb = [&](const std::vector<int>& act, auto Vp, auto KVp, auto kv, bool with_k, double drop) {
        auto g = gemms(act, [&](int b) {
            const int n = items[b].n;
            return GemmItem{Vp(b), n, Vp(b), n, w[b].G, kv(b), kv(b), kv(b), n, 1.0, 0.0};
        }, s);
        gemm_vb(g, true, false, s);
        Batch<SvqbItem> q;
        for (int b : act) q.h.push_back(SvqbItem{w[b].G, kv(b), w[b].dv, w[b].Gd, w[b].ev, w[b].Tq});
        q.sync(s);
        hipLaunchKernelGGL(k_svqb_prep, dim3(q.size()), dim3(256), 0, s, q.d.p);
        launch_check("svqb_prep");
        jacobi(act, [&](int b) { return w[b].G; }, kv, [&](int b) { return w[b].Gd; }, [&](int b) { return w[b].ev; });
        hipLaunchKernelGGL(k_svqb_finish, dim3(q.size()), dim3(256), 0, s, q.d.p, drop);
        launch_check("svqb_finish");
        auto g2 = gemms(act, [&](int b) {
            const int n = items[b].n;
            return GemmItem{Vp(b), n, w[b].Tq, kv(b), w[b].T2, n, n, kv(b), kv(b), 1.0, 0.0};
        }, s);
        gemm_vb(g2, false, false, s);
        copy_block(act, [&](int b) { return w[b].T2; }, Vp, kv);
        if (with_k) {
            auto g3 = gemms(act, [&](int b) {
                const int n = items[b].n;
                return GemmItem{KVp(b), n, w[b].Tq, kv(b), w[b].T2, n, n, kv(b), kv(b), 1.0, 0.0};
            }, s);
            gemm_vb(g3, false, false, s);
            copy_block(act, [&](int b) { return w[b].T2; }, KVp, kv);
        }
    };
    // Rayleigh-Ritz on the first m(b) columns of W (K-images in KW): X := W C,
    // KX := KW C (C = top k eigenvectors), theta; with_p: P := W[:, k:m] C[k:m, :]
    auto rayleigh_ritz = [&](const std::vector<int>& act, auto mcols, bool with_p) {
        auto g = gemms(act, [&](int b) {
            const int n = items[b].n, m = mcols(b);
            return GemmItem{w[b].W, n, w[b].KW, n, w[b].H, m, m, m, n, smallest ? -1.0 : 1.0, 0.0};
        }, s);
        gemm_vb(g, true, false, s);
        if (smallest) {
            Batch<ZeroColItem> zb;
            int mmax = 1;
            for (int b : act) {
                zb.h.push_back(ZeroColItem{w[b].W, items[b].n, mcols(b), w[b].H});
                mmax = std::max(mmax, mcols(b));
            }
            zb.sync(s);
            hipLaunchKernelGGL(k_exclude_zero_cols, dim3(mmax, zb.size()), dim3(256), 0, s, zb.d.p);
            launch_check("lobpcg_zero_cols");
        }
        jacobi(act, [&](int b) { return w[b].H; }, mcols, [&](int b) { return w[b].Ev; },
               [&](int b) { return w[b].ev; });
        // new X and KX into T2 / T1 (n x k each), then P, KP
        auto gx = gemms(act, [&](int b) {
            const int n = items[b].n, m = mcols(b), k = items[b].k;
            return GemmItem{w[b].W, n, w[b].Ev, m, w[b].T2, n, n, k, m, 1.0, 0.0};
        }, s);
        gemm_vb(gx, false, false, s);
        auto gk = gemms(act, [&](int b) {
            const int n = items[b].n, m = mcols(b), k = items[b].k;
            return GemmItem{w[b].KW, n, w[b].Ev, m, w[b].T1, n, n, k, m, 1.0, 0.0};
        }, s);
        gemm_vb(gk, false, false, s);
        if (with_p) {
            auto gp = gemms(act, [&](int b) {
                const int n = items[b].n, m = mcols(b), k = items[b].k;
                return GemmItem{w[b].W + (int64_t)n * k, n, w[b].Ev + k, m, w[b].P, n, n, k, m - k, 1.0, 0.0};
            }, s);
            gemm_vb(gp, false, false, s);
        }
        auto kk = [&](int b) { return items[b].k; };
        copy_block(act, [&](int b) { return w[b].T2; }, [&](int b) { return w[b].W; }, kk);
        copy_block(act, [&](int b) { return w[b].T1; }, [&](int b) { return w[b].KW; }, kk);
        for (int b : act) {
            if (smallest) hipLaunchKernelGGL(k_negate, dim3(1), dim3(64), 0, s, w[b].ev, items[b].theta, items[b].k);
            else DD_HIP(hipMemcpyAsync(items[b].theta, w[b].ev, items[b].k * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        launch_check("lobpcg_theta");
    };

    auto kk = [&](int b) { return items[b].k; };
    std::vector<int> act(nb);
    for (int b = 0; b < nb; ++b) act[b] = b;
    // start: X := orth(X0), KX := K X, Rayleigh-Ritz in span(X)
    copy_block(act, [&](int b) { return items[b].X; }, [&](int b) { return w[b].W; }, kk);
    svqb(act, [&](int b) { return w[b].W; }, [&](int b) { return w[b].KW; }, kk, false, 1e-26);
    apply_op(act, [&](int b) { return w[b].W; }, [&](int b) { return w[b].KW; }, kk);
    rayleigh_ritz(act, kk, false);
    std::vector<char> has_p(nb, 0);
    std::vector<double> best(nb, INFINITY);
    std::vector<int> best_it(nb, 0), stall(nb, 0), restore;
    for (int it = 1; it <= maxit + 1 && !act.empty(); ++it) {
        // residuals R = KX - X theta into W[:, k:2k], norms
        {
            Batch<ResItem> rb;
            int kmax = 1;
            for (int b : act) {
                const int n = items[b].n, k = items[b].k;
                rb.h.push_back(ResItem{w[b].W, w[b].KW, w[b].W + (int64_t)n * k, has_p[b] ? w[b].P : nullptr, n, k,
                                       items[b].theta, w[b].rho});
                kmax = std::max(kmax, k);
            }
            rb.sync(s);
            hipLaunchKernelGGL(k_residual, dim3(kmax, rb.size()), dim3(256), 0, s, rb.d.p, smallest ? 0 : 1, tol);
            launch_check("lobpcg_residual");
        }
        std::vector<int> next;
        for (int b : act) {
            const int k = items[b].k;
            std::vector<double> r(k), th(k);
            d2h(r.data(), w[b].rho, k, s);
            d2h(th.data(), items[b].theta, k, s);
            DD_HIP(hipStreamSynchronize(s));
            // relative residual, less the rounding floor of forming K x (about
            // eps ||K|| ~ eps theta_1 absolute), so a pair at the floor counts as converged
            double worst = 0.0;
            for (int j = 0; j < std::min(items[b].nev, k); ++j) {
                const double floor =
                    (!smallest && th[j] > 0.0) ? 64.0 * 2.220446049250313e-16 * th[0] / th[j] : 0.0;
                worst = std::max(worst, std::max(0.0, r[j] - floor));
            }
            // safeguard: keep the best iterate; stop an item whose residual has not
            // improved for three iterations once within 100 tol, or has grown 1e3-fold
            // over its best (rounding in the basis can drive LOBPCG away once
            // converged), and return the best iterate
            const bool better = worst < best[b];
            if (better) {
                best[b] = worst;
                best_it[b] = it - 1;
                stall[b] = 0;
                DD_HIP(hipMemcpyAsync(w[b].Xb, w[b].W, (size_t)items[b].n * k * sizeof(double), hipMemcpyDeviceToDevice, s));
                DD_HIP(hipMemcpyAsync(w[b].thb, items[b].theta, k * sizeof(double), hipMemcpyDeviceToDevice, s));
            } else {
                stall[b] += 1;
            }
            const bool done = worst <= tol;
            const bool stalled = (stall[b] >= 3 && best[b] <= 100.0 * tol) || worst > 1e3 * best[b] || !(worst == worst);
            st.resid[b] = std::min(worst, best[b]);
            st.iters[b] = better ? it - 1 : best_it[b];
            if (done || stalled) {
                if (!better) restore.push_back(b);
                if (!done && best[b] > 100.0 * tol) st.maxit_hits += 1;
                continue;
            }
            if (it <= maxit) {
                next.push_back(b);
            } else {
                if (!better) restore.push_back(b);
                st.maxit_hits += 1;
            }
        }
        act.swap(next);
        if (act.empty()) break;
        // V = [R, P] at W[:, k:], K-images of P at KW[:, 2k:]
        std::vector<int> a1, a2;  // without / with P
        for (int b : act) (has_p[b] ? a2 : a1).push_back(b);
        for (const auto* grp : {&a1, &a2}) {
            const std::vector<int>& g = *grp;
            if (g.empty()) continue;
            const bool wp = grp == &a2;
            auto kv = [&](int b) { return wp ? 2 * items[b].k : items[b].k; };
            if (wp)
                copy_block(g, [&](int b) { return w[b].P; }, [&](int b) { return w[b].W + (int64_t)2 * items[b].n * items[b].k; }, kk);
            auto Vp = [&](int b) { return w[b].W + (int64_t)items[b].n * items[b].k; };
            auto KVp = [&](int b) { return w[b].KW + (int64_t)items[b].n * items[b].k; };
            if (smallest) {  // R := K R (preconditioned residuals), through T2 as the output
                apply_K(g, Vp, [&](int b) { return w[b].T2; }, kk);
                copy_block(g, [&](int b) { return w[b].T2; }, Vp, kk);
            }
            // project V against X twice: C1 = X^T V, V -= X C1
            for (int pass = 0; pass < 2; ++pass) {
                auto gc = gemms(g, [&](int b) {
                    const int n = items[b].n, k = items[b].k;
                    return GemmItem{w[b].W, n, Vp(b), n, w[b].C1, k, k, kv(b), n, 1.0, 0.0};
                }, s);
                gemm_vb(gc, true, false, s);
                auto gv = gemms(g, [&](int b) {
                    const int n = items[b].n, k = items[b].k;
                    return GemmItem{w[b].W, n, w[b].C1, k, Vp(b), n, n, kv(b), k, -1.0, 1.0};
                }, s);
                gemm_vb(gv, false, false, s);
            }
            // orthonormalise V, then its operator images afresh: an image carried
            // along (as P's could be) holds an absolute rounding of about eps ||K||,
            // which normalising a nearly converged (tiny) direction would inflate
            svqb(g, Vp, KVp, kv, false, 1e-8);
            apply_op(g, Vp, KVp, kv);
            rayleigh_ritz(g, [&](int b) { return items[b].k + kv(b); }, true);
            for (int b : g) has_p[b] = 1;
        }
    }
    // items stopped past their best iterate get it back
    for (int b : restore) {
        DD_HIP(hipMemcpyAsync(w[b].W, w[b].Xb, (size_t)items[b].n * items[b].k * sizeof(double), hipMemcpyDeviceToDevice, s));
        DD_HIP(hipMemcpyAsync(items[b].theta, w[b].thb, items[b].k * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    // Ritz vectors out
    std::vector<int> all(nb);
    for (int b = 0; b < nb; ++b) all[b] = b;
    copy_block(all, [&](int b) { return w[b].W; }, [&](int b) { return items[b].X; }, kk);
    DD_HIP(hipStreamSynchronize(s));
}

}  // namespace dd
