// Batched dense linear algebra on uneven items (FP64), gfx950.
#pragma once
#include "common.hpp"

namespace dd {

// Column-major matrix view: element (r, c) at p[r + c*ld].
template <class T>
struct MatT {
    T* p;
    int ld;
    int m;
    int n;
};
using DMat = MatT<double>;
using FMat = MatT<float>;

// A batch of per-item descriptors with host and device copies.
template <class T>
struct Batch {
    std::vector<T> h;
    DBuf<T> d;
    void sync(hipStream_t s) {
        d.alloc(h.size());
        h2d(d.p, h.data(), h.size(), s);
        DD_HIP(hipStreamSynchronize(s));
    }
    int size() const { return (int)h.size(); }
};

// QR storage: A (m x n, m >= n) holds R above and the Householder vectors below
// the diagonal (unit diagonal implicit); tau[n]; T holds one 32x32 upper
// triangular compact-WY factor per 32-column panel (qr_t_size); G holds the
// Gram matrix V^T V of every 128-column block of reflectors (qr_g_size); W is
// scratch of qr_w_size(max columns of the matrices the reflectors touch).
// zrow, zslope (optional structure): column j of A has zeros in rows
// > zrow + zslope * j, as for a stack [X; I] (zrow = rows of X, zslope = 1) or
// for [T; I] with T upper triangular and the rows interleaved t_0, i_0, t_1,
// i_1, ... (zrow = 1, zslope = 2).  Householder steps keep the structure, so
// reflector j vanishes below row zrow + zslope * j too and every step only
// touches rows <= zrow + zslope * (last column of the block).
constexpr int QR_NOZ = 1 << 29;
struct QRItem {
    DMat A;
    double* tau;
    double* T;
    double* W;
    int wld;   // unused (kept for layout stability)
    int nfac;  // factor only the first nfac columns (<= n); the rest receive Q^T
    double* G;
    int zrow = QR_NOZ;
    int zslope = 1;
};

// Application of the Q stored in V (m x k reflectors, T and G as above) to C
// (m x nc, rows aligned with V's rows).
struct ORItem {
    DMat V;   // m x k: reflector j in column j, rows j..m-1
    double* T;
    DMat C;
    double* W;  // qr_w_size(C.n)
    double* G;
    int zrow = QR_NOZ;  // reflector j is zero below row zrow + zslope * j
    int zslope = 1;
};
// rows touched by the reflectors in columns [c0, c0 + w) of an m-row matrix
// rows that columns [c0, c0 + w) can have nonzero: up to row zrow + zslope * (c0 + w - 1)
__host__ __device__ inline int qr_rows(int m, int zrow, int zslope, int c0, int w) {
    const int64_t r = (int64_t)zrow + (int64_t)zslope * (c0 + w - 1) + 1;
    return r < m ? (int)r : m;
}

constexpr int QR_NB = 32;   // inner panel width
constexpr int QR_OB = 128;  // outer block (four inner panels)
constexpr int CH_NB = 64;
inline int64_t qr_t_size(int k) { return (int64_t)((k + QR_NB - 1) / QR_NB) * QR_NB * QR_NB; }
constexpr int QR_PAIR = 256; // two outer blocks applied to C in one pass
// G: the Gram matrix of every 128-column block, then the cross Gram V_b^T V_a
// of every 256-column pair (a, b) of blocks
inline int64_t qr_g_size(int k) {
    return ((int64_t)(k + QR_OB - 1) / QR_OB + (k + QR_PAIR - 1) / QR_PAIR) * QR_OB * QR_OB;
}
inline int64_t qr_w_size(int ncols) { return (int64_t)QR_PAIR * ncols; }

// C := alpha * op(A) op(B) + beta * C for every item (dims from C and A).
struct GemmItem {
    const double* A;
    int lda;
    const double* B;
    int ldb;
    double* C;
    int ldc;
    int M, N, K;
    double alpha, beta;
};

void gemm_vb(Batch<GemmItem>& g, bool ta, bool tb, hipStream_t s);
// C := alpha A A^T + beta C, lower-triangle tiles only (A = M x K, B unused)
void syrk_vb(Batch<GemmItem>& g, hipStream_t s);
// C := alpha A B + beta C with A upper triangular (M = K, zeros stored below)
void gemm_upper_a_vb(Batch<GemmItem>& g, hipStream_t s);

// In-place lower Cholesky A = L L^T (upper triangle untouched).  A may be a
// tall panel (m >= n): the rows below the leading n x n block are solved
// against L^T (supernodal panel factorisation).  info[b] = 1-based column of
// the first non-positive pivot (0 if none).
void potrf_vb(Batch<DMat>& A, int* dinfo, hipStream_t s);
// The same in FP32 (FP32 MFMA products with FP32 accumulation).  info[b] also
// records a positive pivot below piv_min (the factor is then too inaccurate
// for the caller's use): the 1-based column of the first such pivot.
void potrf_vb(Batch<FMat>& A, int* dinfo, float piv_min, hipStream_t s);

// B := L^{-1} B (trans = false) or L^{-T} B (trans = true), L lower (only the
// lower triangle of L is read).  Item b: L[b] (n x n), B[b] (n x nrhs).
void trsm_vb(Batch<DMat>& L, Batch<DMat>& B, bool trans, hipStream_t s, bool lower_rhs = false);
void trsm_vb(Batch<FMat>& L, Batch<FMat>& B, bool trans, hipStream_t s, bool lower_rhs = false);

// Householder QR in place (first nfac columns factored, all columns updated).
void geqrf_vb(Batch<QRItem>& q, hipStream_t s);
// C := Q C (trans = false) or Q^T C (trans = true).
void ormqr_vb(Batch<ORItem>& o, bool trans, hipStream_t s);
// C := Q [I; 0] for C preset to the identity (explicit Q, orgqr-style cost)
void orgqr_vb(Batch<ORItem>& o, hipStream_t s);
// T and G factors for reflectors stored in V with taus (used after sytrd).
void build_t_vb(Batch<ORItem>& o, const std::vector<double*>& htau, hipStream_t s);

// Householder tridiagonalisation of symmetric A, in place.  Only the lower
// triangle of A is read (the strict upper triangle may hold anything and is
// overwritten with garbage).  d[n], e[n-1] (off-diagonal), tau[n-1];
// reflector k stored in A[k+1:, k] with an explicit 1 at row k+1.
constexpr int TRD_NB = 32;  // panel width of the blocked tridiagonalisation
// partial sums of the lower-triangle matrix-vector product: row partials of
// every 64-column block (T x n), then column partials of every chunk of
// TRD_RB row blocks below each column block (at most T x T x 64), T = ceil(n / 64)
constexpr int TRD_RB = 4;
__host__ __device__ inline int64_t trd_part_size(int n) {
    const int64_t T = (n + 63) / 64;
    return T * n + T * T * 64;
}
struct TriItem {
    DMat A;
    double* d;
    double* e;
    double* tau;
    double* part;  // >= ceil(n / 256) doubles
    double* p;     // n doubles
    double* W;     // n x TRD_NB (ld n)
    double* aux;   // 2 * TRD_NB doubles
    double* yp;    // trd_part_size(n) doubles
};
void sytrd_vb(Batch<TriItem>& t, hipStream_t s);

// Eigenvalues of the tridiagonal (d, e) below `thr`, ascending, at most cap:
// count[b] written, mu[0..count).
struct EigItem {
    const double* d;
    const double* e;
    int n;
    double* mu;
    int* count;
    int cap;
    double thr;
};
void stebz_vb(Batch<EigItem>& e, hipStream_t s);

// Eigenvectors of the tridiagonal for the eigenvalues mu[0..count) by inverse
// iteration (three rounds); after every round the vectors of each cluster
// (consecutive eigenvalues closer than cluster_tol * ||T||) are
// orthonormalised together by Householder QR.  Y: n x count (ld >= n).
// hmu: host copies of the eigenvalues (cluster detection).
struct VecItem {
    const double* d;
    const double* e;
    int n;
    const double* mu;
    const int* count;
    double* Y;
    int ldy;
    double* work;  // stein_work_size(n, number of eigenvalues) doubles
};
inline int64_t stein_work_size(int n, int count) {
    return (int64_t)4 * n * 256 * std::max<int64_t>(1, (count + 255) / 256);
}
void stein_vb(Batch<VecItem>& v, const std::vector<std::vector<double>>& hmu, double cluster_tol, hipStream_t s);

// Local solves with explicit triangular inverses: x := W^T (W x) for W lower
// triangular n x n (column-major, exact zeros above the diagonal), one vector
// per item.  y (n) and part (trmv_part_size(n)) are per-item workspaces.
template <class TW>
struct TrmvItemT {
    const TW* W;
    int ld;
    int n;
    double* x;
    double* y;
    double* part;
};
using TrmvItem = TrmvItemT<double>;
using TrmvItem32 = TrmvItemT<float>;  // FP32 factor, FP32 arithmetic, FP64 vectors
constexpr int TRMV_RB = 64;    // rows per tile of y = W x
constexpr int TRMV_CC = 512;   // columns per partial sum of y = W x
inline int64_t trmv_part_size(int n) { return (int64_t)((n + TRMV_CC - 1) / TRMV_CC) * n; }
// tiles of x = W^T y: 16 columns by a chunk of TRMV_CC rows at or below their diagonal block
__host__ __device__ inline int trmv_t_tiles(int n) {
    const int ng = (n + 15) / 16, nch = (n + TRMV_CC - 1) / TRMV_CC;
    int t = 0;
    for (int c = 0; c < nch; ++c) t += min(ng, (TRMV_CC / 16) * (c + 1));
    return t;
}
void trinv_apply_vb(Batch<TrmvItem>& t, hipStream_t s);
void trinv_apply_vb(Batch<TrmvItem32>& t, hipStream_t s);
void trmv_n_vb(Batch<TrmvItem>& t, hipStream_t s);  // y := W x   (uses part)
void trmv_t_vb(Batch<TrmvItem>& t, hipStream_t s);  // x := W^T y
// Absolute column sums colsum[b][j] = sum_i |A_ij| and row sums rowsum[b][i]
// (for ||A||_1, ||A||_inf, hence the bound ||A||_2 <= sqrt(||A||_1 ||A||_inf))
void abs_sums_vb(Batch<DMat>& A, double* const* colsum, double* const* rowsum, hipStream_t s);
// FP64 -> FP32 copy of n elements; *bad is set to 1 if a rounded value is not finite
void to_fp32(const double* src, float* dst, int64_t n, int* bad, hipStream_t s);

// FP32 local factors with symmetric Jacobi scaling.  Item: A (n x n FP64,
// lower triangle read), d (n FP64), A32 (n x n FP32), W32 (n x n FP32),
// bad (one flag per item).
struct Fp32Item {
    const double* A;
    double* d;
    float* A32;
    float* W32;
    int n;
    int* bad;
};
// d_k = a_kk^{-1/2} (1 where a_kk <= 0: the FP64 factor reports that), then
// A32 = fl32(D A D) on the lower triangle and zero above
void jacobi_fp32_vb(Batch<Fp32Item>& f, hipStream_t s);
// W32 := I
void identity_fp32_vb(Batch<Fp32Item>& f, hipStream_t s);
// W32 := W32 D (column j times d_j, lower triangle); bad = 1 if an entry is
// not finite
void scale_cols_fp32_vb(Batch<Fp32Item>& f, hipStream_t s);
// B (n x k FP64, ld n) <-> B32 (n x k FP32, ld n) with the rows scaled by d:
// to32: B32 = fl32(d o B); otherwise B = d o B32
struct RowScaleItem {
    double* B;
    float* B32;
    const double* d;
    int n, k;
};
void rowscale_fp32_vb(Batch<RowScaleItem>& r, bool to32, hipStream_t s);

// Elementwise helpers.
void set_identity_vb(Batch<DMat>& A, double diag, hipStream_t s);  // A := diag * I (m x n)
// S (2n x n) := [sc_b X^T ; I] with rows interleaved (row 2i: sc_b X^T row i, row
// 2i+1: identity row i), X n x n (item b of X, S), scale per item on the device
void stack_interleaved_vb(Batch<DMat>& X, Batch<DMat>& S, const double* dscale, hipStream_t s);
// D (2n x n) := the rows of Q (2n x n) de-interleaved: D[i] = Q[2i], D[n + i] = Q[2i + 1]
void deinterleave_rows_vb(Batch<DMat>& Q, Batch<DMat>& D, hipStream_t s);
void copy_vb(Batch<DMat>& src, Batch<DMat>& dst, bool transpose, double scale, hipStream_t s);
void add_diag_vb(Batch<DMat>& A, const double* dshift, hipStream_t s);  // A(i,i) += shift[b]
void symmetrize_vb(Batch<DMat>& A, hipStream_t s);                     // A := (A + A^T)/2
void zero_upper_vb(Batch<DMat>& A, hipStream_t s);                     // strictly upper := 0
void zero_lower_vb(Batch<DMat>& A, hipStream_t s);                     // strictly lower := 0
void axpby_vb(Batch<DMat>& X, Batch<DMat>& Y, const double* dalpha, const double* dbeta, hipStream_t s);  // Y := a X + b Y
void frob_vb(Batch<DMat>& A, double* dout, hipStream_t s);             // out[b] = ||A||_F
// Largest eigenvalue of symmetric H[b] by Lanczos with full
// reorthogonalisation (at most K <= 128 steps).  work[b] (device pointer
// array) holds n*(K+2) + 2*(K+1) + 1 doubles; dout[b] = eigenvalue;
// dflag[b] is scratch (set to 1 once the item has converged).
void lanczos_max_vb(Batch<DMat>& H, double* const* work, int K, double* dout, int* dflag, hipStream_t s);

}  // namespace dd
