// Block eigensolver for the local eigenproblem (3.3) in cap mode: LOBPCG
// (Knyazev 2001) for the largest eigenvalues of the symmetric positive definite
// K = M^T M, batched over the subdomains of a level, plus the batched dense
// symmetric eigensolver (two-sided Jacobi) its Rayleigh-Ritz steps use.
#pragma once
#include "dense.hpp"

namespace dd {

// ---------------------------------------------------------------------------
// Batched symmetric eigensolver for small matrices (m <= JAC_MAX): cyclic
// two-sided Jacobi with the round-robin ordering (disjoint rotations applied
// together), one workgroup per item with the matrix in LDS.  A (m x m, only
// (A + A^T)/2 is used) -> eigenvalues w[0..m) in descending order and the
// orthonormal eigenvectors as the columns of V (m x m, same order).
// ---------------------------------------------------------------------------
constexpr int JAC_MAX = 128;
struct JacItem {
    const double* A;
    int lda;
    int m;
    double* V;
    int ldv;
    double* w;
};
void jacobi_eig_vb(Batch<JacItem>& b, hipStream_t s);

// ---------------------------------------------------------------------------
// LOBPCG.  Explicit mode: the largest eigenvalues of K = M^T M with an explicit
// lower triangular M (n x n).  Matrix-free mode: the smallest eigenvalues of
// S~ = K^{-1} = L^{-1} RL RL^T L^{-T} (L, RL lower triangular n x n), applied
// through the factors (solves with L, products with RL: backward stable),
// preconditioned by K = L^T RL^{-T} RL^{-1} L, also through the factors (its
// rounding, of order eps cond(RL)^2, only slows the iteration); nothing n x n
// is formed.  Converged pairs are soft-locked (their residual and P direction
// leave the basis).  X (n x k, ld n) holds the start block on entry and the
// Ritz vectors on exit, ordered from the wanted end (theta descending for K,
// ascending for S~, i.e. the reciprocal values ascending in both).
// ---------------------------------------------------------------------------
struct LobItem {
    int n, k, nev;
    const double* M;   // explicit mode
    int ldm;
    const double* L;   // matrix-free mode
    int ldl;
    const double* RL;
    int ldr;
    double* X;
    double* theta;     // k (device)
};
struct LobStats {
    std::vector<int> iters;      // per item
    std::vector<double> resid;   // per item: max relative residual of the nev wanted pairs at exit
    int maxit_hits = 0;
};
// Stops an item once its nev leading pairs have ||K x_j - theta_j x_j|| <=
// (tol + 64 eps theta_1 / theta_j) theta_j (explicit; the second term is the
// rounding floor of forming K x, about eps ||K||) or ||S~ x_j - theta_j x_j||
// <= tol (matrix-free; ||S~|| <= 1), or after maxit iterations.
void lobpcg_vb(std::vector<LobItem>& items, bool matrix_free, double tol, int maxit, hipStream_t s, LobStats& st);

// Orthonormal basis of the columns of V (m x kv, ld m, kv <= JAC_MAX) by SVQB:
// Q = V T with V^T V = U Lambda U^T, T = D U Lambda^{-1/2} (D the column
// scaling), directions with lambda <= 1e-13 lambda_max dropped (zero columns).
struct OrthItem {
    const double* V;
    int m, kv;
    double* Q;   // m x kv, ld m
};
void orth_basis_vb(std::vector<OrthItem>& items, hipStream_t s);

// Gaussian block from a counter-based generator: X[b](r, c) = N(0,1) from
// SplitMix64(seed_b, r + c * n) by the Box-Muller transform.
struct RandItem {
    double* X;
    int ld, m, n;
    uint64_t seed;
};
void gaussian_vb(Batch<RandItem>& b, hipStream_t s);

// X[:, j] := X[:, j] / ||X[:, j]|| + eps G[:, j] / ||G[:, j]|| for j < k (X, G: n x k,
// ld n); a zero column of X becomes G's.  Keeps a structured start block full rank.
struct MixItem {
    double* X;
    const double* G;
    int n, k;
    double eps;
};
void mix_random_vb(Batch<MixItem>& b, hipStream_t s);

// mu[b][j] = ||Y[b](:, j)||^2 for j < n (column norms squared).
struct ColItem {
    const double* Y;
    int ld, m, n;
    double* out;
};
void colnorm2_vb(Batch<ColItem>& b, hipStream_t s);

}  // namespace dd
