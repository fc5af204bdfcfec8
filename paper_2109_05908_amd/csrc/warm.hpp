// Learned start blocks for the block eigensolver of (3.3): features of the
// boundary layer Delta_i computed from A alone, a small network (MLP) that maps
// them to a weight per boundary node, its training kernels, and the sparse
// products of the start block A_ii^{-1} A(Omega_i, Delta_i) diag(w) G.
#pragma once
#include "dense.hpp"
#include "sparse.hpp"

namespace dd {

constexpr int WS_F = 8;   // features per boundary node
constexpr int WS_H = 32;  // hidden width (two tanh layers)
constexpr int WS_P = WS_F * WS_H + WS_H + WS_H * WS_H + WS_H + WS_H + 1;  // parameters

// Index maps of one level as the kernels need them (device pointers).  For
// subdomain i: ext[offE[i] ..] = [I_i, Gamma_i, Delta_i], each ascending, with
// counts[3i..3i+2] = |I_i|, |Gamma_i|, |Delta_i|.
struct WsMaps {
    CsrDev A;
    int N;
    const int64_t* offE;
    const int32_t* counts;
    const int32_t* ext;
};

// per-subdomain mean of log a_rr over Omega_i: smean[N]
void ws_subdomain_logdiag(const WsMaps& M, double* smean, hipStream_t s);
// features of every boundary node (rows offD[i] + a, a < |Delta_i|), row-major x WS_F
void ws_features(const WsMaps& M, const double* smean, const int64_t* offD, int64_t total, double* feats,
                 hipStream_t s);

// B_i (n_i x k, ld n_i, rows in Omega_i order) = A(Omega_i, Delta_i) diag(w_i) G_i, with
// G_i (|Delta_i| x k, ld |Delta_i|) and w_i (|Delta_i|, or all ones when w is null) at
// offset offD[i]; B[i], G[i] device pointers.
void ws_range_product(const WsMaps& M, const int64_t* offO, int64_t rows, const int64_t* offD, const double* w,
                      double* const* G, double* const* B, const int32_t* kcols, hipStream_t s);
// Gt_i (|Delta_i| x p_i) = A(Omega_i, Delta_i)^T U_i, U_i (n_i x p_i, ld n_i)
void ws_adjoint_product(const WsMaps& M, const int64_t* offD, int64_t total, double* const* U, double* const* Gt,
                        const int32_t* pcols, hipStream_t s);
// out[r] = ||Q(r, :)||^2 * scale for the rows of a batch of Q (m x n, ld)
struct RowItem {
    const double* Q;
    int ld, m, n;
    double* out;
    double scale;
};
void ws_row_leverage(Batch<RowItem>& b, hipStream_t s);

// ---- the network ---------------------------------------------------------
// params: W1 (WS_H x WS_F, row-major), b1, W2 (WS_H x WS_H), b2, w3 (WS_H), b3;
// inputs standardised by mean/stdv (WS_F each); output w = softplus(o).
void mlp_forward(const double* params, const double* mean, const double* stdv, const double* feats, int64_t n,
                 double* out, hipStream_t s);
// loss = sum_s c_s (w_s - t_s)^2 and its gradient (WS_P) into grad, loss into *dloss (device)
void mlp_loss_grad(const double* params, const double* mean, const double* stdv, const double* feats,
                   const double* target, const double* weight, int64_t n, double* grad, double* dloss,
                   hipStream_t s);
// Adam (Kingma & Ba 2015) step t >= 1 on WS_P parameters
void mlp_adam(double* params, const double* grad, double* m1, double* m2, double lr, int t, hipStream_t s);

// feature statistics over n samples: mean and standard deviation per feature (device, WS_F each)
void ws_feature_stats(const double* feats, int64_t n, double* mean, double* stdv, hipStream_t s);

}  // namespace dd
