// Host orchestration of the setup (Sec. 2-3 of the paper), the two-level
// additive Schwarz apply (2.1) and PCG, behind the C-ABI of include/dd.h.
#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "bchol.hpp"
#include "mrhs.hpp"
#include "coarse.hpp"
#include "lobpcg.hpp"
#include "warm.hpp"

namespace dd {

constexpr double kEps = 2.220446049250313e-16;  // 2^-52, the shift's epsilon

// ---------------------------------------------------------------------------
// per-item arenas
// ---------------------------------------------------------------------------
template <class T>
struct ArenaT {
    DBuf<T> buf;
    std::vector<T*> ptr;
    void alloc(const std::vector<int64_t>& sizes) {
        std::vector<int64_t> off(sizes.size() + 1, 0);
        for (size_t i = 0; i < sizes.size(); ++i) off[i + 1] = off[i] + ((std::max<int64_t>(sizes[i], 1) + 31) / 32) * 32;
        buf.alloc(off.back());
        ptr.resize(sizes.size());
        for (size_t i = 0; i < sizes.size(); ++i) ptr[i] = buf.p + off[i];
    }
    void release() { buf.release(); ptr.clear(); }
};
using Arena = ArenaT<double>;
using ArenaF = ArenaT<float>;

struct Timer {
    hipStream_t s;
    std::chrono::steady_clock::time_point t0;
    explicit Timer(hipStream_t st) : s(st) { t0 = std::chrono::steady_clock::now(); }
    double lap() {
        DD_HIP(hipStreamSynchronize(s));
        auto t1 = std::chrono::steady_clock::now();
        double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        t0 = t1;
        return ms;
    }
};

struct Model;  // warm-start network (warm.hip)
struct Opts {
    int local_prec = DD_FP64;
    int select = DD_SEL_THRESHOLD;
    int nev_cap = 0;
    int validate = 0;
    int coarsen = 64;
    int schwarz = DD_SCHWARZ_ADDITIVE;
    int eig_solver = DD_EIG_DENSE;
    int lobpcg_maxit = 100;
    double lobpcg_tol = 1e-8;
    bool lobpcg_tol_set = false;
    int warm_start = DD_START_RANDOM;
    uint64_t seed = 0;
    const void* model = nullptr;
    int graph_pcg = 0;
};

// dd_options -> Opts; DD_ERR_INVALID_ARG for values out of range
static int parse_opts(const dd_options* o, Opts& out) {
    if (!o) return DD_OK;
    if (o->local_prec != DD_FP64 && o->local_prec != DD_FP32) return DD_ERR_INVALID_ARG;
    if (o->select != DD_SEL_THRESHOLD && o->select != DD_SEL_THRESHOLD_CAP) return DD_ERR_INVALID_ARG;
    if (o->select == DD_SEL_THRESHOLD_CAP && o->nev_cap < 0) return DD_ERR_INVALID_ARG;
    if (o->schwarz != DD_SCHWARZ_ADDITIVE && o->schwarz != DD_SCHWARZ_DEFLATED) return DD_ERR_INVALID_ARG;
    if (o->eig_solver < DD_EIG_DENSE || o->eig_solver > DD_EIG_LOBPCG_MATFREE) return DD_ERR_INVALID_ARG;
    // the block solver computes the nev_cap wanted pairs of the cap mode (1..32 per subdomain)
    if (o->eig_solver != DD_EIG_DENSE && (o->select != DD_SEL_THRESHOLD_CAP || o->nev_cap < 1 || o->nev_cap > 32))
        return DD_ERR_INVALID_ARG;
    if (o->lobpcg_maxit < 0 || !(o->lobpcg_tol >= 0.0)) return DD_ERR_INVALID_ARG;
    if (o->warm_start < DD_START_RANDOM || o->warm_start > DD_START_MODEL) return DD_ERR_INVALID_ARG;
    out.local_prec = o->local_prec;
    out.select = o->select;
    out.nev_cap = o->nev_cap;
    out.validate = o->validate;
    if (o->coarsen > 0) out.coarsen = o->coarsen;
    out.schwarz = o->schwarz;
    out.eig_solver = o->eig_solver;
    if (o->lobpcg_maxit > 0) out.lobpcg_maxit = o->lobpcg_maxit;
    if (o->lobpcg_tol > 0.0) {
        out.lobpcg_tol = o->lobpcg_tol;
        out.lobpcg_tol_set = true;
    }
    out.warm_start = o->warm_start;
    out.seed = o->seed;
    out.model = o->warm_start_model;
    if (o->graph_pcg < 0 || o->graph_pcg > 64) return DD_ERR_INVALID_ARG;
    out.graph_pcg = o->graph_pcg;
    return DD_OK;
}

// Workspace of right-preconditioned GMRES on one level: Krylov basis V
// (n x (restart + 1)), the preconditioned directions M v_j (n x restart), a
// vector, the partial sums of V^T w and the device and pinned host copies of a
// Hessenberg column.
constexpr int kMaxRestart = 64;
constexpr int kGemvBlocks = 256;
constexpr int kHcol = 2 * (kMaxRestart + 1) + 1;  // first pass, second pass, ||w||^2
struct GmresWork {
    int cap = 0;
    int64_t n = 0;
    DBuf<double> V, Zf, w, part, h;
    double* hp = nullptr;
    GmresWork() = default;
    GmresWork(const GmresWork&) = delete;
    GmresWork& operator=(const GmresWork&) = delete;
    ~GmresWork() {
        if (hp) (void)hipHostFree(hp);
    }
    void ensure(int64_t nn, int restart) {
        if (nn == n && restart <= cap) return;
        const int c = std::max(restart, cap);
        V.alloc((size_t)nn * (c + 1));
        Zf.alloc((size_t)nn * c);
        w.alloc(nn);
        part.alloc((size_t)kGemvBlocks * (kMaxRestart + 1));
        h.alloc(kHcol + kMaxRestart);
        if (!hp) DD_HIP(hipHostMalloc(&hp, (kHcol + kMaxRestart) * sizeof(double)));
        cap = c;
        n = nn;
    }
};

enum Phase { PH_SETS, PH_EXTRACT, PH_CHOL, PH_QR, PH_POLAR, PH_SIGMA, PH_SCHUR, PH_EIG, PH_BASIS, PH_E, PH_EFACT, PH_OTHER };
static const char* kPhaseNames[DD_NPHASE] = {"sets+maps", "extract", "local_cholesky", "qr_X", "polar_qdwh",
                                             "sigma1", "schur_qr", "eigen", "basis", "assemble_E", "factor_E",
                                             "other"};

// ---------------------------------------------------------------------------
// one decomposed level
// ---------------------------------------------------------------------------
struct Level {
    // matrix of this level (owned copy)
    int64_t n = 0, nnz = 0;
    DBuf<int32_t> rowptr, colind;
    DBuf<double> val;
    CsrDev A() const { return CsrDev{n, nnz, rowptr.p, colind.p, val.p}; }

    int N = 0, delta = 1;
    double tau = 0.0;
    DBuf<int32_t> part;
    std::vector<int32_t> hcounts;  // 3N
    DBuf<int32_t> counts;
    std::vector<int64_t> hoffE, hoffO, hoffI;
    DBuf<int64_t> offE, offO, offI;
    DBuf<int32_t> ext, omega_flat, ilocal;
    DBuf<int64_t> memb_ptr, memb;
    std::vector<int> ni, nt, nI, nG, nD;

    Arena L;  // local Cholesky factors (n_i x n_i, lower); released after setup
    Arena W;  // explicit inverses W_i = L_i^{-1} (lower), used by the apply
    ArenaF W32;  // FP32 form: W_i = Lhat_i^{-1} D_i from the FP32 factor of D_i A_ii D_i
    bool fp32 = false;  // the FP32 form (subdomains that fell back keep an FP64 W_i)
    // FP32 form, during the setup only: the FP32 factors Lhat_i, the scales d_i
    // (offsets hoffO) and which subdomains fell back to FP64
    ArenaF L32;
    DBuf<double> jd;
    std::vector<int> fp64;
    std::vector<int> p;
    std::vector<int32_t> status;
    DBuf<int32_t> pcnt;
    std::vector<int64_t> hoffC;
    DBuf<int64_t> offC;
    Arena Z;
    DBuf<double*> dZ;
    std::vector<std::vector<double>> mu;
    std::vector<double> sigma1;
    std::vector<int> lob_iters;      // block eigensolver: iterations and final residual per subdomain
    std::vector<double> lob_resid;
    int64_t nC = 0;
    BlockChol E;                // block-sparse Cholesky factor of the coarse operator
    std::vector<double> Ecopy;  // small coarse operators only (inspection)
    std::vector<uint8_t> hadj;  // block graph of E: hadj[i*N+j] = 1 iff A(Omega_Ii, Omega_Ij) != 0, i != j

    // batch of independent systems (dd_setup_batch): the subdomains
    // [hsub[j], hsub[j+1]) of system j; on levels >= 1 also its dofs
    // [hseg[j], hseg[j+1]) and the system of every dof (level 0 keeps these in
    // the handle)
    std::vector<int32_t> hsub;
    std::vector<int64_t> hseg;
    DBuf<int64_t> dseg;
    DBuf<int32_t> seg_id;

    // Krylov workspace for systems with this level's matrix
    DBuf<double> kr, kz, kp, kq, kro, kx;
    GmresWork gm;
    DBuf<double> dy, dt;  // deflated apply: coarse correction and the residual it leaves

    // apply workspace
    DBuf<double> rloc, yloc, tpart, yC;
    Batch<TrmvItem> Tb;
    Batch<TrmvItem32> Tb32;

    SubInfo sub() const {
        return SubInfo{N, counts.p, offE.p, offO.p, ext.p, part.p, ilocal.p, pcnt.p, offC.p, dZ.p};
    }
};

// A PCG iteration captured as a HIP graph (two-level additive handles), replayed
// in batches of at most `chunk` between host checks; the scalars live on the
// device, slots below
enum GSlot { G_RZ, G_PQ, G_ALPHA, G_RN2, G_RZN, G_BETA, G_THR, G_ITS, G_STATE, G_MAXIT, G_NSLOT };
struct GraphPcg {
    int chunk = 0;
    int ns = 1;                // systems (a batch handle: one set of slots per system, S[slot * ns + k])
    hipStream_t cs = nullptr;  // capture stream (default priority)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DBuf<double> S;            // G_NSLOT x ns device scalars
    double* hS = nullptr;      // pinned copy
    GraphPcg() = default;
    GraphPcg(const GraphPcg&) = delete;
    GraphPcg& operator=(const GraphPcg&) = delete;
    ~GraphPcg() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
        if (hS) (void)hipHostFree(hS);
    }
};
// Several right-hand sides in lockstep: the same scalars per column, slot-major
// (S[slot * kMrhs + k]), and column-blocked work vectors of the finest level.
struct BlockPcg {
    DBuf<double> S, r, z, p, q;   // S: G_NSLOT x kMrhs; vectors: kMrhs x n
    DBuf<double> rloc, yloc, tpart, yC;  // kMrhs copies of the level's apply workspaces
    Batch<TrmvMItem<double>> Tm;
    Batch<TrmvMItem<float>> Tm32;
    double* hS = nullptr;          // pinned copy of S
    BlockPcg() = default;
    BlockPcg(const BlockPcg&) = delete;
    BlockPcg& operator=(const BlockPcg&) = delete;
    ~BlockPcg() {
        if (hS) (void)hipHostFree(hS);
    }
};

struct Handle {
    std::unique_ptr<GraphPcg> gp;
    std::unique_ptr<BlockPcg> bp;  // several right-hand sides in lockstep (dd_pcg, dd_apply)
    std::vector<std::unique_ptr<Level>> lv;
    int32_t levels_req = 2;  // levels asked for at setup
    Opts opt;
    dd_info_t info{};
    // dot-product scratch
    DBuf<double> partial, dots;
    double* hpin = nullptr;
    // batch of independent systems (dd_setup_batch): dof offsets of the
    // systems in the block-diagonal union, the system of every dof, and the
    // per-system Krylov scalars (pinned host, device)
    std::vector<int64_t> sys_off;
    DBuf<int64_t> dsys_off;
    DBuf<int32_t> sys_id;
    std::vector<int32_t> sub_off;  // subdomains of each system on level 0
    DBuf<double> dscal;
    double* hscal = nullptr;
    int nsys() const { return sys_off.size() > 1 ? (int)sys_off.size() - 1 : 1; }
    ~Handle() {
        if (hpin) (void)hipHostFree(hpin);
        if (hscal) (void)hipHostFree(hscal);
    }
};

// ---------------------------------------------------------------------------
// QDWH scalar weights (Nakatsukasa, Bai & Gygi 2010)
// ---------------------------------------------------------------------------
// An iteration takes the QR form while c > kQdwhQrWeight and the Cholesky form
// after.  The Cholesky form's error grows like c times the unit roundoff
// (Nakatsukasa & Higham 2012), about 4e-12 at this bound, which leaves H
// accurate far beyond what the local eigenvalues and the apply need; the
// customary bound of 100 would keep the second iteration (c between about 200
// and 1e4 for l0 from 1e-6 to 1e-10) in the QR form, at 8.7 n^3 flops instead
// of 3.3 n^3.
constexpr double kQdwhQrWeight = 2e4;

static void qdwh_weights(double l, double& a, double& b, double& c) {
    const double l2 = l * l;
    const double g = std::cbrt(4.0 * (1.0 - l2) / (l2 * l2));
    a = std::sqrt(1.0 + g) + 0.5 * std::sqrt(8.0 - 4.0 * g + 8.0 * (2.0 - l2) / (l2 * std::sqrt(1.0 + g)));
    b = (a - 1.0) * (a - 1.0) / 4.0;
    c = a + b - 1.0;
}

template <class T>
static std::vector<T> to_host(const T* d, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    d2h(h.data(), d, n, s);
    DD_HIP(hipStreamSynchronize(s));
    return h;
}

static Batch<DMat> mats(const std::vector<double*>& p, const std::vector<int>& ld, const std::vector<int>& m,
                        const std::vector<int>& n, hipStream_t s, const std::vector<int>* active = nullptr) {
    Batch<DMat> b;
    for (size_t i = 0; i < p.size(); ++i)
        if (!active || (*active)[i]) b.h.push_back(DMat{p[i], ld[i], m[i], n[i]});
    b.sync(s);
    return b;
}

// ---------------------------------------------------------------------------
// setup of one level: sets, local splittings, eigenproblems, coarse space
// ---------------------------------------------------------------------------
static void build_e_csr(Level& Lv, Level& next, hipStream_t s);

// a1 and a2 of one level: the ordered sets I, Gamma, Delta and the index maps
// (Sec. 2), then the dense blocks Y_i = X_i^T (n~_i x n_i) into Y and A_ii
// (n_i x n_i) into Lv.L (Sec. 3.1, (3.1)).
static void sets_and_extract(Level& Lv, dd_info_t& info, Timer& tm, Arena& Y, hipStream_t s) {
    const int N = Lv.N;
    const int delta = Lv.delta;
    const int64_t n = Lv.n;
    const CsrDev A = Lv.A();

    // ---- a1: sets and index maps -------------------------------------------------
    overlap_sets(A, Lv.part.p, N, delta, Lv.hcounts, Lv.ext, s);
    Lv.nI.resize(N); Lv.nG.resize(N); Lv.nD.resize(N); Lv.ni.resize(N); Lv.nt.resize(N);
    Lv.hoffE.assign(N + 1, 0); Lv.hoffO.assign(N + 1, 0); Lv.hoffI.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) {
        Lv.nI[i] = Lv.hcounts[3 * i];
        Lv.nG[i] = Lv.hcounts[3 * i + 1];
        Lv.nD[i] = Lv.hcounts[3 * i + 2];
        Lv.ni[i] = Lv.nI[i] + Lv.nG[i];
        Lv.nt[i] = Lv.ni[i] + Lv.nD[i];
        Lv.hoffE[i + 1] = Lv.hoffE[i] + Lv.nt[i];
        Lv.hoffO[i + 1] = Lv.hoffO[i] + Lv.ni[i];
        Lv.hoffI[i + 1] = Lv.hoffI[i] + Lv.nI[i];
    }
    Lv.counts = upload(Lv.hcounts, s);
    Lv.offE = upload(Lv.hoffE, s);
    Lv.offO = upload(Lv.hoffO, s);
    Lv.offI = upload(Lv.hoffI, s);
    membership(Lv.offE.p, Lv.offO.p, Lv.counts.p, Lv.ext.p, N, n, Lv.memb_ptr, Lv.memb, Lv.hoffO[N], s);
    Lv.omega_flat.alloc(Lv.hoffO[N]);
    Lv.ilocal.alloc(n);
    omega_flatten(N, Lv.offE.p, Lv.offO.p, Lv.counts.p, Lv.ext.p, Lv.hoffO[N], Lv.omega_flat.p, Lv.ilocal.p, s);
    info.phase_ms[PH_SETS] += tm.lap();

    const auto& ni = Lv.ni;
    const auto& nt = Lv.nt;

    // ---- a2: dense Y_i = X_i^T and A_ii ------------------------------------------------
    {
        std::vector<int64_t> sy(N), sa(N);
        for (int i = 0; i < N; ++i) {
            sy[i] = (int64_t)nt[i] * ni[i];
            sa[i] = (int64_t)ni[i] * ni[i];
        }
        Y.alloc(sy);
        Lv.L.alloc(sa);
        fill(Y.buf.p, Y.buf.n, 0.0, s);
        fill(Lv.L.buf.p, Lv.L.buf.n, 0.0, s);
        DBuf<double*> dY(N), dA(N);
        h2d(dY.p, Y.ptr.data(), N, s);
        h2d(dA.p, Lv.L.ptr.data(), N, s);
        extract(A, N, Lv.offE.p, Lv.offO.p, Lv.counts.p, Lv.ext.p, dY.p, dA.p, Lv.hoffO[N], s);
        DD_HIP(hipStreamSynchronize(s));
    }
    info.phase_ms[PH_EXTRACT] += tm.lap();
}

// ---------------------------------------------------------------------------
// warm-start network (a dd_model)
// ---------------------------------------------------------------------------
struct Model {
    DBuf<double> params, mean, stdv, m1, m2, grad, dloss;
    DBuf<double> feats, target, weight;  // training samples (device)
    int64_t ns = 0;                      // samples stored
    int nsub = 0;                        // subdomains they came from
    int step = 0;                        // Adam steps taken
    bool stats = false;                  // mean / stdv fixed
    Model() {
        params.alloc(WS_P); m1.alloc(WS_P); m2.alloc(WS_P); grad.alloc(WS_P); dloss.alloc(1);
        mean.alloc(WS_F); stdv.alloc(WS_F);
    }
};

static WsMaps ws_maps(const Level& Lv) {
    return WsMaps{Lv.A(), Lv.N, Lv.offE.p, Lv.counts.p, Lv.ext.p};
}

// Start blocks of the block eigensolver, X_i (n_Ii x k_i) into Yev.  Random: a
// Gaussian block.  Range / model: by the near-kernel characterisation of the
// splitting (its kernel is A_ii^{-1} A(Omega_i, Delta_i) applied to data on
// Delta_i), X_i = L_I^T [A_ii^{-1} A(Omega_i, Delta_i) diag(w) G]_I with G
// Gaussian on Delta_i and w = 1 (range) or the network's weight of every
// boundary node (model); L_I^T maps the pencil's vectors to those of the
// reciprocal form.  A subdomain with fewer boundary nodes than columns takes
// the random block.
static void start_blocks(Level& Lv, const Opts& opt, const std::vector<int>& kb, Arena& Yev, hipStream_t s) {
    const int N = Lv.N;
    const auto& ni = Lv.ni;
    const auto& nI = Lv.nI;
    const auto& nD = Lv.nD;
    const Model* model = static_cast<const Model*>(opt.model);
    const bool structured = opt.warm_start == DD_START_RANGE || (opt.warm_start == DD_START_MODEL && model);
    std::vector<int> rnd(N, 1);
    if (structured)
        for (int i = 0; i < N; ++i) rnd[i] = nD[i] < kb[i];
    auto item_seed = [&](int i, uint64_t salt) {
        return opt.seed * 0x9E3779B97F4A7C15ull + (uint64_t)Lv.n * 0x100000001B3ull + (uint64_t)i * 2654435761ull + salt;
    };
    {
        Batch<RandItem> rb;
        for (int i = 0; i < N; ++i)
            if (rnd[i]) rb.h.push_back(RandItem{Yev.ptr[i], nI[i], nI[i], kb[i], item_seed(i, 0)});
        if (rb.size()) {
            rb.sync(s);
            gaussian_vb(rb, s);
        }
    }
    if (!structured) return;
    std::vector<int> act(N);
    for (int i = 0; i < N; ++i) act[i] = !rnd[i];
    std::vector<int64_t> hoffD(N + 1, 0);
    for (int i = 0; i < N; ++i) hoffD[i + 1] = hoffD[i] + nD[i];
    const int64_t totD = hoffD[N];
    if (!totD) return;
    DBuf<int64_t> offD = upload(hoffD, s);
    const WsMaps M = ws_maps(Lv);
    DBuf<double> w;
    if (opt.warm_start == DD_START_MODEL) {
        DBuf<double> smean(N), feats((size_t)totD * WS_F);
        w.alloc(totD);
        ws_subdomain_logdiag(M, smean.p, s);
        ws_features(M, smean.p, offD.p, totD, feats.p, s);
        mlp_forward(model->params.p, model->mean.p, model->stdv.p, feats.p, totD, w.p, s);
        DD_HIP(hipStreamSynchronize(s));
    }
    Arena G, B;
    std::vector<int64_t> sg(N), sb(N);
    for (int i = 0; i < N; ++i) {
        sg[i] = (int64_t)std::max(1, nD[i]) * kb[i];
        sb[i] = (int64_t)ni[i] * kb[i];
    }
    G.alloc(sg);
    B.alloc(sb);
    {
        Batch<RandItem> rb;
        for (int i = 0; i < N; ++i)
            if (act[i]) rb.h.push_back(RandItem{G.ptr[i], nD[i], nD[i], kb[i], item_seed(i, 0x5bd1e995ull)});
        rb.sync(s);
        gaussian_vb(rb, s);
    }
    DBuf<double*> dG(N), dB(N);
    h2d(dG.p, G.ptr.data(), N, s);
    h2d(dB.p, B.ptr.data(), N, s);
    std::vector<int32_t> kc(N);
    for (int i = 0; i < N; ++i) kc[i] = act[i] ? kb[i] : 0;  // random items: no columns
    DBuf<int32_t> dk = upload(kc, s);
    ws_range_product(M, Lv.offO.p, Lv.hoffO[N], offD.p, w.p, dG.p, dB.p, dk.p, s);
    // U = A_ii^{-1} B by the local Cholesky factor (FP32 form: D Lhat^{-T} Lhat^{-1} D
    // by the FP32 factor, ample for a start block), then X = L_I^T U_I
    std::vector<int> a64(N), a32(N);
    for (int i = 0; i < N; ++i) {
        a32[i] = act[i] && Lv.fp32 && !Lv.fp64[i];
        a64[i] = act[i] && !a32[i];
    }
    {
        Batch<DMat> Lb = mats(Lv.L.ptr, ni, ni, ni, s, &a64);
        Batch<DMat> Bb = mats(B.ptr, ni, ni, kb, s, &a64);
        if (Bb.size()) {
            trsm_vb(Lb, Bb, false, s);
            trsm_vb(Lb, Bb, true, s);
        }
    }
    if (std::count(a32.begin(), a32.end(), 1)) {
        ArenaF B32;
        std::vector<int64_t> s32(N);
        for (int i = 0; i < N; ++i) s32[i] = a32[i] ? (int64_t)ni[i] * kb[i] : 1;
        B32.alloc(s32);
        Batch<RowScaleItem> rs;
        Batch<FMat> Lf, Bf;
        for (int i = 0; i < N; ++i) {
            if (!a32[i]) continue;
            rs.h.push_back(RowScaleItem{B.ptr[i], B32.ptr[i], Lv.jd.p + Lv.hoffO[i], ni[i], kb[i]});
            Lf.h.push_back(FMat{Lv.L32.ptr[i], ni[i], ni[i], ni[i]});
            Bf.h.push_back(FMat{B32.ptr[i], ni[i], ni[i], kb[i]});
        }
        rs.sync(s);
        Lf.sync(s);
        Bf.sync(s);
        rowscale_fp32_vb(rs, true, s);
        trsm_vb(Lf, Bf, false, s);
        trsm_vb(Lf, Bf, true, s);
        rowscale_fp32_vb(rs, false, s);
        DD_HIP(hipStreamSynchronize(s));
    }
    Batch<GemmItem> g;
    for (int i = 0; i < N; ++i)
        if (act[i]) g.h.push_back(GemmItem{Lv.L.ptr[i], ni[i], B.ptr[i], ni[i], Yev.ptr[i], nI[i], nI[i], kb[i], nI[i], 1.0, 0.0});
    g.sync(s);
    gemm_vb(g, true, false, s);
    // a weighted block can be numerically rank-deficient (weight on a few boundary
    // nodes, or an exactly zero column): every column gets a Gaussian component of
    // relative size 1e-10, above the level at which the start block's
    // orthonormalisation drops a direction (1e-13), so the block stays full rank
    // while its useful directions are untouched
    Arena Gr;
    std::vector<int64_t> sr(N);
    for (int i = 0; i < N; ++i) sr[i] = act[i] ? (int64_t)nI[i] * kb[i] : 1;
    Gr.alloc(sr);
    {
        Batch<RandItem> rb;
        Batch<MixItem> mb;
        for (int i = 0; i < N; ++i) {
            if (!act[i]) continue;
            rb.h.push_back(RandItem{Gr.ptr[i], nI[i], nI[i], kb[i], item_seed(i, 0x27d4eb2full)});
            mb.h.push_back(MixItem{Yev.ptr[i], Gr.ptr[i], nI[i], kb[i], 1e-10});
        }
        rb.sync(s);
        mb.sync(s);
        gaussian_vb(rb, s);
        mix_random_vb(mb, s);
    }
    DD_HIP(hipStreamSynchronize(s));
}

// (3.3) in cap mode by the block solver.  With Boolean D_i the wanted pairs are
// the nev smallest mu of S~ = L_I^{-1} S_I L_I^{-T} (reciprocal form), i.e. the
// nev largest lambda of K = S~^{-1}.  The QR of the permuted factor was taken
// over every column, so S_I = R_II^T R_II with R_II upper triangular, and
// K = M^T M with M = R_II^{-T} L_I (lower triangular): either formed (one
// triangular solve) or, matrix-free, applied as L_I^T R_II^{-1} R_II^{-T} L_I.
// The largest lambda are well separated (they grow like 1/s towards the near
// kernel), so LOBPCG on K converges in a few iterations.  The kept mu are the
// Rayleigh quotients of S~ itself, mu_j = ||R_II L_I^{-T} y_j||^2, which are
// accurate to eps in absolute terms (the lambda form only to eps ||K||).
// Output as the dense route's: Yev (n_Ii x p_i, orthonormal, mu ascending),
// Lv.p, Lv.mu.
static void eigen_lobpcg(Level& Lv, const Opts& opt, dd_info_t& info, Arena& Fp, const std::vector<int>& nc,
                         Arena& Yev, hipStream_t s) {
    const int N = Lv.N;
    const auto& nt = Lv.nt;
    const auto& ni = Lv.ni;
    const auto& nI = Lv.nI;
    const bool mf = opt.eig_solver == DD_EIG_LOBPCG_MATFREE;
    const int nev = opt.nev_cap;
    constexpr int kGuard = 8;  // block size nev + 8: the guard vectors speed up the last wanted pairs
    std::vector<int> kb(N);
    std::vector<int64_t> sI2(N), sk(N), skk(N);
    for (int i = 0; i < N; ++i) {
        kb[i] = std::min(nI[i], nev + kGuard);
        sI2[i] = (int64_t)nI[i] * nI[i];
        sk[i] = (int64_t)nI[i] * kb[i];
        skk[i] = kb[i];
    }
    // RL = R_II^T (lower); R_II sits at rows and columns [nc, nt) of the factored Fp
    Arena RL;
    RL.alloc(sI2);
    {
        std::vector<double*> rii(N);
        for (int i = 0; i < N; ++i) rii[i] = Fp.ptr[i] + nc[i] + (int64_t)nc[i] * nt[i];
        Batch<DMat> Rsrc = mats(rii, nt, nI, nI, s);
        Batch<DMat> Rb = mats(RL.ptr, nI, nI, nI, s);
        copy_vb(Rsrc, Rb, true, 1.0, s);
        zero_upper_vb(Rb, s);  // the reflectors below R_II's diagonal land above RL's
        DD_HIP(hipStreamSynchronize(s));
    }
    Fp.release();
    Batch<DMat> LI = mats(Lv.L.ptr, ni, nI, nI, s);
    Batch<DMat> RLb = mats(RL.ptr, nI, nI, nI, s);
    Arena Mx;
    if (!mf) {
        Mx.alloc(sI2);
        Batch<DMat> Mb = mats(Mx.ptr, nI, nI, nI, s);
        copy_vb(LI, Mb, false, 1.0, s);
        trsm_vb(RLb, Mb, false, s, true);  // M = RL^{-1} L_I, lower triangular
    }
    // start blocks
    Yev.alloc(sk);
    start_blocks(Lv, opt, kb, Yev, s);
    Arena th;
    th.alloc(skk);
    std::vector<LobItem> items(N);
    for (int i = 0; i < N; ++i)
        items[i] = LobItem{nI[i], kb[i], std::min(nev, kb[i]), mf ? nullptr : Mx.ptr[i], nI[i], Lv.L.ptr[i], ni[i],
                           RL.ptr[i], nI[i], Yev.ptr[i], th.ptr[i]};
    LobStats st;
    // the matrix-free form tests an absolute residual of S~ (norm <= 1): a tighter default
    const double tol = (mf && !opt.lobpcg_tol_set) ? 1e-12 : opt.lobpcg_tol;
    lobpcg_vb(items, mf, tol, opt.lobpcg_maxit, s, st);
    Mx.release();
    info.eig_maxit_hits += st.maxit_hits;
    Lv.lob_iters = st.iters;
    Lv.lob_resid = st.resid;
    // mu_j = ||R_II L_I^{-T} y_j||^2
    Arena T1, T2, mu;
    T1.alloc(sk);
    T2.alloc(sk);
    mu.alloc(skk);
    {
        Batch<DMat> Ys = mats(Yev.ptr, nI, nI, kb, s), Tb = mats(T1.ptr, nI, nI, kb, s);
        copy_vb(Ys, Tb, false, 1.0, s);
        trsm_vb(LI, Tb, true, s);
        Batch<GemmItem> g;
        for (int i = 0; i < N; ++i)
            g.h.push_back(GemmItem{RL.ptr[i], nI[i], T1.ptr[i], nI[i], T2.ptr[i], nI[i], nI[i], kb[i], nI[i], 1.0, 0.0});
        g.sync(s);
        gemm_vb(g, true, false, s);
        Batch<ColItem> cb;
        for (int i = 0; i < N; ++i) cb.h.push_back(ColItem{T2.ptr[i], nI[i], nI[i], kb[i], mu.ptr[i]});
        cb.sync(s);
        colnorm2_vb(cb, s);
    }
    const auto hmu = to_host(mu.buf.p, mu.buf.n, s);
    Lv.p.assign(N, 0);
    Lv.mu.assign(N, {});
    for (int i = 0; i < N; ++i) {
        const double* m = hmu.data() + (mu.ptr[i] - mu.buf.p);
        int p = 0;
        while (p < std::min(nev, kb[i]) && m[p] < Lv.tau) ++p;  // prefix: mu ascending, keep mu < tau
        Lv.p[i] = p;
        Lv.mu[i].assign(m, m + p);
    }
}

// `next` (nullable): when given, E is not factored but handed to the next
// level as its CSR matrix (multilevel recursion).
static void build_level(Level& Lv, const Opts& opt, dd_info_t& info, hipStream_t s, Level* next) {
    Timer tm(s);
    const int N = Lv.N;
    const CsrDev A = Lv.A();
    Arena Y;
    sets_and_extract(Lv, info, tm, Y, s);
    const bool lob = opt.eig_solver != DD_EIG_DENSE;
    const auto& ni = Lv.ni;
    const auto& nt = Lv.nt;
    const auto& nI = Lv.nI;
    std::vector<int> nc(N);
    for (int i = 0; i < N; ++i) nc[i] = nt[i] - nI[i];

    // ---- a4: local Cholesky A_ii = L_i L_i^T (exact subdomain solver) -------------------
    // FP32 form: D_i A_ii D_i (d_k = a_kk^{-1/2}) is rounded to FP32 and factored
    // Lhat_i Lhat_i^T on FP32 MFMA with FP32 accumulation, and W_i = Lhat_i^{-1} D_i
    // is formed (W_i^T W_i = A_ii^{-1}).  A subdomain whose FP32 factor meets a
    // pivot at or below n_max eps_32 (the rounding level of the scaled entries:
    // the factor would carry no digits) or whose W_i is not finite falls back to
    // FP64.  The FP64 factor is then needed only for its leading block L_I (the
    // eigenproblem), except for the subdomains that fell back; the start blocks
    // solve with the FP32 factor.  All of this is decided before the FP64
    // factorisation overwrites A_ii.
    const bool f32 = opt.local_prec == DD_FP32;
    Lv.fp64.assign(N, 1);
    Lv.fp32 = f32;
    if (f32) {
        std::vector<int64_t> sa(N);
        int nmax = 0;
        for (int i = 0; i < N; ++i) {
            sa[i] = (int64_t)ni[i] * ni[i];
            nmax = std::max(nmax, ni[i]);
        }
        Lv.L32.alloc(sa);
        Lv.W32.alloc(sa);
        Lv.jd.alloc(std::max<int64_t>(1, Lv.hoffO[N]));
        DBuf<int32_t> fbad(N), finfo(N);
        DD_HIP(hipMemsetAsync(fbad.p, 0, N * sizeof(int32_t), s));
        DD_HIP(hipMemsetAsync(finfo.p, 0, N * sizeof(int32_t), s));
        Batch<Fp32Item> fb;
        Batch<FMat> Lf, Wf;
        for (int i = 0; i < N; ++i) {
            fb.h.push_back(Fp32Item{Lv.L.ptr[i], Lv.jd.p + Lv.hoffO[i], Lv.L32.ptr[i], Lv.W32.ptr[i], ni[i], fbad.p + i});
            Lf.h.push_back(FMat{Lv.L32.ptr[i], ni[i], ni[i], ni[i]});
            Wf.h.push_back(FMat{Lv.W32.ptr[i], ni[i], ni[i], ni[i]});
        }
        fb.sync(s);
        Lf.sync(s);
        Wf.sync(s);
        jacobi_fp32_vb(fb, s);
        potrf_vb(Lf, finfo.p, (float)nmax * FLT_EPSILON, s);
        identity_fp32_vb(fb, s);
        trsm_vb(Lf, Wf, false, s, true);
        scale_cols_fp32_vb(fb, s);
        const auto hi = to_host(finfo.p, N, s), hb = to_host(fbad.p, N, s);
        for (int i = 0; i < N; ++i) {
            Lv.fp64[i] = (hi[i] != 0 || hb[i] != 0) ? 1 : 0;
            info.fp32_fallbacks += Lv.fp64[i];
        }
    }
    {
        // FP64: the whole A_ii, or its leading block A_I where the FP32 factor stands
        std::vector<int> mf(N);
        for (int i = 0; i < N; ++i) mf[i] = Lv.fp64[i] ? ni[i] : nI[i];
        Batch<DMat> Ab = mats(Lv.L.ptr, ni, mf, mf, s);
        DBuf<int32_t> dinfo(N);
        DD_HIP(hipMemsetAsync(dinfo.p, 0, N * sizeof(int32_t), s));
        potrf_vb(Ab, dinfo.p, s);
        zero_upper_vb(Ab, s);
        auto hinfo = to_host(dinfo.p, N, s);
        for (int i = 0; i < N; ++i)
            DD_CHECK(hinfo[i] == 0, DD_ERR_NOT_SPD, "local block A_ii is not positive definite");
    }
    info.phase_ms[PH_CHOL] += tm.lap();

    // ---- a3 (part 1): Householder QR of Y_i = X_i^T --------------------------------------
    Arena qtau, qT, qW, qG;
    {
        std::vector<int64_t> st(N), sT(N), sW(N), sG(N);
        for (int i = 0; i < N; ++i) {
            st[i] = ni[i];
            sT[i] = qr_t_size(ni[i]);
            sW[i] = qr_w_size(std::max(ni[i], nt[i]));
            sG[i] = qr_g_size(ni[i]);
        }
        qtau.alloc(st);
        qT.alloc(sT);
        qW.alloc(sW);
        qG.alloc(sG);
        Batch<QRItem> qb;
        for (int i = 0; i < N; ++i)
            qb.h.push_back(QRItem{DMat{Y.ptr[i], nt[i], nt[i], ni[i]}, qtau.ptr[i], qT.ptr[i], qW.ptr[i], QR_NB, ni[i], qG.ptr[i]});
        qb.sync(s);
        geqrf_vb(qb, s);
    }
    info.phase_ms[PH_QR] += tm.lap();

    // ---- a3 (part 2): polar factor of R by QDWH; H = (R R^T)^{1/2} -------------------------
    // R (ni x ni upper) from the QR; the iterate is kept transposed, Xt_0 = R^T / alpha.
    Arena Rm, Xt, Wk;
    std::vector<int64_t> sq(N), s4(N);
    for (int i = 0; i < N; ++i) {
        sq[i] = (int64_t)ni[i] * ni[i];
        s4[i] = 4 * sq[i];
    }
    Rm.alloc(sq);
    Xt.alloc(sq);
    Wk.alloc(s4);
    std::vector<int> two_ni(N);
    for (int i = 0; i < N; ++i) two_ni[i] = 2 * ni[i];
    {
        std::vector<double*> ytop(Y.ptr);
        Batch<DMat> Ysrc = mats(ytop, nt, ni, ni, s);
        Batch<DMat> Rb = mats(Rm.ptr, ni, ni, ni, s);
        Batch<DMat> Xb = mats(Xt.ptr, ni, ni, ni, s);
        copy_vb(Ysrc, Rb, false, 1.0, s);
        zero_lower_vb(Rb, s);
        copy_vb(Rb, Xb, true, 1.0, s);  // Xt = R^T (lower)
        // alpha >= ||R||_2 and l0 <= sigma_min(R) / alpha from norm bounds of R and R^{-1}
        DBuf<double> dnorm(N), dnorm2(N);
        frob_vb(Rb, dnorm.p, s);
        std::vector<double*> wfirst(Wk.ptr);
        Batch<DMat> Ib = mats(wfirst, ni, ni, ni, s);
        set_identity_vb(Ib, 1.0, s);
        trsm_vb(Xb, Ib, false, s, true);  // R^{-T}
        frob_vb(Ib, dnorm2.p, s);
        auto alpha = to_host(dnorm.p, N, s);
        auto rinv = to_host(dnorm2.p, N, s);
        // tighter guaranteed bounds: ||M||_2 <= sqrt(||M||_1 ||M||_inf) for M = R and R^{-1}
        // (a larger l0 saves QR-based iterations; it must stay <= sigma_min / alpha)
        {
            Arena cs, rs;
            std::vector<int64_t> sz(ni.begin(), ni.end());
            cs.alloc(sz);
            rs.alloc(sz);
            DBuf<double*> dcs(N), drs(N);
            h2d(dcs.p, cs.ptr.data(), N, s);
            h2d(drs.p, rs.ptr.data(), N, s);
            auto norm_1inf = [&](Batch<DMat>& M, std::vector<double>& out) {
                abs_sums_vb(M, dcs.p, drs.p, s);
                const auto hc = to_host(cs.buf.p, cs.buf.n, s);
                const auto hr = to_host(rs.buf.p, rs.buf.n, s);
                for (int i = 0; i < N; ++i) {
                    const int64_t o = cs.ptr[i] - cs.buf.p;
                    double m1 = 0.0, mi = 0.0;
                    for (int k = 0; k < ni[i]; ++k) {
                        m1 = std::max(m1, hc[o + k]);
                        mi = std::max(mi, hr[o + k]);
                    }
                    out[i] = std::min(out[i], std::sqrt(m1 * mi));
                }
            };
            norm_1inf(Rb, alpha);
            norm_1inf(Ib, rinv);
        }
        std::vector<double> ell(N), inv_alpha(N), zero(N, 0.0);
        for (int i = 0; i < N; ++i) {
            DD_CHECK(alpha[i] > 0 && std::isfinite(rinv[i]), DD_ERR_NOT_SPD, "singular local block row X_i");
            ell[i] = std::min(1.0, 0.9 / (alpha[i] * rinv[i]));
            inv_alpha[i] = 1.0 / alpha[i];
        }
        DBuf<double> da = upload(inv_alpha, s), dz0 = upload(zero, s);
        axpby_vb(Xb, Xb, da.p, dz0.p, s);  // Xt := Xt / alpha

        const bool verbose = std::getenv("DD_VERBOSE") != nullptr;
        if (verbose) {
            std::vector<double> e2(ell);
            std::sort(e2.begin(), e2.end());
            fprintf(stderr, "dd: qdwh l0 min %.3e median %.3e max %.3e\n", e2.front(), e2[N / 2], e2.back());
        }
        std::vector<int> done(N, 0);
        for (int it = 0; it < 20; ++it) {
            std::vector<int> actQ(N, 0), actC(N, 0);
            std::vector<double> ca(N), cb(N), cc(N), coefQ(N), beta(N), coefC(N);
            int anyQ = 0, anyC = 0;
            for (int i = 0; i < N; ++i) {
                if (done[i]) continue;
                double a, b, c;
                qdwh_weights(ell[i], a, b, c);
                ca[i] = a; cb[i] = b; cc[i] = c;
                beta[i] = b / c;
                if (c > kQdwhQrWeight) { actQ[i] = 1; anyQ = 1; coefQ[i] = (a - b / c) / std::sqrt(c); }
                else { actC[i] = 1; anyC = 1; coefC[i] = a - b / c; }
            }
            if (!anyQ && !anyC) break;
            if (verbose) {
                int nq = 0, nch = 0;
                for (int i = 0; i < N; ++i) { nq += actQ[i]; nch += actC[i]; }
                fprintf(stderr, "dd: qdwh iteration %d: %d QR-based, %d Cholesky-based\n", it, nq, nch);
            }
            if (anyQ) {
                // S = [sqrt(c) Xt^T ; I]  (2 ni x ni), QR, explicit Q = [Q1; Q2]; Xt := b/c Xt + coef Q2 Q1^T
                std::vector<double*> sp(N), qp(N), scr(N);
                for (int i = 0; i < N; ++i) { sp[i] = Wk.ptr[i]; qp[i] = Wk.ptr[i] + 2 * sq[i]; }
                Batch<DMat> Xq = mats(Xt.ptr, ni, ni, ni, s, &actQ);
                std::vector<double*> stop(sp), sbot(N);
                for (int i = 0; i < N; ++i) sbot[i] = sp[i] + ni[i];
                Batch<DMat> Stop = mats(stop, two_ni, ni, ni, s, &actQ);
                Batch<DMat> Sbot = mats(sbot, two_ni, ni, ni, s, &actQ);
                std::vector<double> sqc(N, 0.0);
                for (int i = 0; i < N; ++i) sqc[i] = actQ[i] ? std::sqrt(cc[i]) : 0.0;
                // The first iterate Xt = R^T / alpha is lower triangular, so S = [sqrt(c) Xt^T; I]
                // is [upper triangular; I]: with its rows interleaved, column j is zero below row
                // 2j + 1 and the QR and the explicit Q only touch rows up to about 2 (block end)
                // instead of ni + (block end).  Later iterates are full.
                const bool tri = it == 0;
                std::vector<double> sa, sz;
                for (int i = 0; i < N; ++i) if (actQ[i]) { sa.push_back(sqc[i]); sz.push_back(0.0); }
                DBuf<double> dsc = upload(sa, s), dzero = upload(sz, s);
                Batch<DMat> Sfull = mats(sp, two_ni, two_ni, ni, s, &actQ);
                if (tri) {
                    stack_interleaved_vb(Xq, Sfull, dsc.p, s);
                } else {
                    // top = sqrt(c) * Xt^T : copy transposed then scale per item
                    copy_vb(Xq, Stop, true, 1.0, s);
                    axpby_vb(Stop, Stop, dsc.p, dzero.p, s);
                    set_identity_vb(Sbot, 1.0, s);
                }
                const int zr = tri ? 1 : 0, zs = tri ? 2 : 1;
                Arena tq, tT, tW, tG;
                std::vector<int64_t> a1(N), a2(N), a3(N), a4(N);
                for (int i = 0; i < N; ++i) {
                    a1[i] = actQ[i] ? ni[i] : 1;
                    a2[i] = actQ[i] ? qr_t_size(ni[i]) : 1;
                    a3[i] = actQ[i] ? qr_w_size(ni[i]) : 1;
                    a4[i] = actQ[i] ? qr_g_size(ni[i]) : 1;
                }
                tq.alloc(a1); tT.alloc(a2); tW.alloc(a3); tG.alloc(a4);
                Batch<QRItem> qb;
                Batch<ORItem> ob;
                for (int i = 0; i < N; ++i) {
                    if (!actQ[i]) continue;
                    // [sqrt(c) Xt^T; I]: column j is zero below row ni + j (interleaved: 1 + 2j)
                    const int zrow = tri ? zr : ni[i];
                    qb.h.push_back(QRItem{DMat{sp[i], 2 * ni[i], 2 * ni[i], ni[i]}, tq.ptr[i], tT.ptr[i], tW.ptr[i], QR_NB, ni[i], tG.ptr[i], zrow, zs});
                    ob.h.push_back(ORItem{DMat{sp[i], 2 * ni[i], 2 * ni[i], ni[i]}, tT.ptr[i], DMat{qp[i], 2 * ni[i], 2 * ni[i], ni[i]}, tW.ptr[i], tG.ptr[i], zrow, zs});
                }
                qb.sync(s);
                ob.sync(s);
                geqrf_vb(qb, s);
                Batch<DMat> Qb = mats(qp, two_ni, two_ni, ni, s, &actQ);
                set_identity_vb(Qb, 1.0, s);
                orgqr_vb(ob, s);
                // Q = [Q1; Q2] (interleaved: de-interleaved into the reflector storage, now free)
                const std::vector<double*>& qsrc = tri ? sp : qp;
                if (tri) deinterleave_rows_vb(Qb, Sfull, s);
                Batch<GemmItem> g;
                for (int i = 0; i < N; ++i) {
                    if (!actQ[i]) continue;
                    g.h.push_back(GemmItem{qsrc[i] + ni[i], 2 * ni[i], qsrc[i], 2 * ni[i], Xt.ptr[i], ni[i], ni[i], ni[i],
                                           ni[i], coefQ[i], beta[i]});
                }
                g.sync(s);
                gemm_vb(g, false, true, s);
                DD_HIP(hipStreamSynchronize(s));
            }
            if (anyC) {
                // Zc = I + c Xt Xt^T = L L^T; W = Zc^{-1} Xt; Xt := b/c Xt + (a - b/c) W
                std::vector<double*> zp(N), wp(N);
                for (int i = 0; i < N; ++i) { zp[i] = Wk.ptr[i]; wp[i] = Wk.ptr[i] + sq[i]; }
                Batch<DMat> Zb = mats(zp, ni, ni, ni, s, &actC);
                Batch<DMat> Wb = mats(wp, ni, ni, ni, s, &actC);
                Batch<DMat> Xc = mats(Xt.ptr, ni, ni, ni, s, &actC);
                set_identity_vb(Zb, 1.0, s);
                Batch<GemmItem> g;
                for (int i = 0; i < N; ++i) {
                    if (!actC[i]) continue;
                    g.h.push_back(GemmItem{Xt.ptr[i], ni[i], Xt.ptr[i], ni[i], zp[i], ni[i], ni[i], ni[i], ni[i], cc[i], 1.0});
                }
                g.sync(s);
                syrk_vb(g, s);  // lower triangle of Zc: all potrf reads
                DBuf<int32_t> dinfo(Zb.size());
                DD_HIP(hipMemsetAsync(dinfo.p, 0, Zb.size() * sizeof(int32_t), s));
                potrf_vb(Zb, dinfo.p, s);
                copy_vb(Xc, Wb, false, 1.0, s);
                trsm_vb(Zb, Wb, false, s);
                trsm_vb(Zb, Wb, true, s);
                std::vector<double> al, be;
                for (int i = 0; i < N; ++i) if (actC[i]) { al.push_back(coefC[i]); be.push_back(beta[i]); }
                DBuf<double> d1 = upload(al, s), d2 = upload(be, s);
                axpby_vb(Wb, Xc, d1.p, d2.p, s);
                auto hinfo = to_host(dinfo.p, Zb.size(), s);
                for (auto v : hinfo) DD_CHECK(v == 0, DD_ERR_EIG, "polar iteration: Cholesky breakdown");
            }
            for (int i = 0; i < N; ++i) {
                if (done[i]) continue;
                const double l = ell[i];
                ell[i] = l * (ca[i] + cb[i] * l * l) / (1.0 + cc[i] * l * l);
                if (std::fabs(1.0 - ell[i]) < 1e-14) done[i] = 1;
            }
            if (it == 19) info.eig_maxit_hits += 1;
        }
        // H = R * Xt_inf  (= R U_p^T, U_p the polar factor of R), symmetrised, in Wk[0:sq]
        Batch<GemmItem> g;
        for (int i = 0; i < N; ++i)
            g.h.push_back(GemmItem{Rm.ptr[i], ni[i], Xt.ptr[i], ni[i], Wk.ptr[i], ni[i], ni[i], ni[i], ni[i], 1.0, 0.0});
        g.sync(s);
        gemm_upper_a_vb(g, s);  // R is upper triangular
        Batch<DMat> Hb = mats(Wk.ptr, ni, ni, ni, s);
        symmetrize_vb(Hb, s);
        DD_HIP(hipStreamSynchronize(s));
    }
    Rm.release();
    Xt.release();
    info.phase_ms[PH_POLAR] += tm.lap();

    // ---- shift s_i = sigma_1i * eps, sigma_1 = lambda_max(H) by Lanczos -------------------
    std::vector<double> shift(N);
    {
        Batch<DMat> Hb = mats(Wk.ptr, ni, ni, ni, s);
        Arena lw;
        std::vector<int64_t> sl(N);
        const int K = 128;
        for (int i = 0; i < N; ++i) sl[i] = (int64_t)ni[i] * (K + 2) + 2 * (K + 1) + 1;
        lw.alloc(sl);
        DBuf<double*> dlw(N);
        h2d(dlw.p, lw.ptr.data(), N, s);
        DBuf<double> dsig(N);
        DBuf<int32_t> dsteps(N);
        lanczos_max_vb(Hb, dlw.p, K, dsig.p, dsteps.p, s);
        Lv.sigma1 = to_host(dsig.p, N, s);
        for (int i = 0; i < N; ++i) shift[i] = Lv.sigma1[i] * kEps;
        DBuf<double> dsh = upload(shift, s);
        add_diag_vb(Hb, dsh.p, s);
        DBuf<int32_t> dinfo(N);
        DD_HIP(hipMemsetAsync(dinfo.p, 0, N * sizeof(int32_t), s));
        potrf_vb(Hb, dinfo.p, s);  // H + sI = L_H L_H^T
        zero_upper_vb(Hb, s);
        auto hinfo = to_host(dinfo.p, N, s);
        for (auto v : hinfo) DD_CHECK(v == 0, DD_ERR_EIG, "shifted square root not positive definite");
    }
    info.phase_ms[PH_SIGMA] += tm.lap();

    // ---- (3.2): F^T = Q_full blkdiag(L_H, sqrt(s) I); Fp = F[:, [c, I]]; QR -> R_II -----------
    Arena Fp;
    {
        Arena Ft;
        std::vector<int64_t> sf(N);
        for (int i = 0; i < N; ++i) sf[i] = (int64_t)nt[i] * nt[i];
        Ft.alloc(sf);
        fill(Ft.buf.p, Ft.buf.n, 0.0, s);
        Batch<DMat> Hb = mats(Wk.ptr, ni, ni, ni, s);
        Batch<DMat> Ftop = mats(Ft.ptr, nt, ni, ni, s);
        copy_vb(Hb, Ftop, false, 1.0, s);
        {
            std::vector<double*> bot(N);
            std::vector<int> nd(N);
            std::vector<int> act(N);
            std::vector<double> sqs;
            for (int i = 0; i < N; ++i) {
                bot[i] = Ft.ptr[i] + ni[i] + (int64_t)ni[i] * nt[i];
                nd[i] = Lv.nD[i];
                act[i] = nd[i] > 0;
                if (act[i]) sqs.push_back(std::sqrt(shift[i]));
            }
            Batch<DMat> Bt = mats(bot, nt, nd, nd, s, &act);
            if (Bt.size()) {
                set_identity_vb(Bt, 1.0, s);
                std::vector<double> z0(sqs.size(), 0.0);
                DBuf<double> d1 = upload(sqs, s), d2 = upload(z0, s);
                axpby_vb(Bt, Bt, d1.p, d2.p, s);
            }
        }
        Wk.release();
        Batch<ORItem> ob;
        for (int i = 0; i < N; ++i)
            ob.h.push_back(ORItem{DMat{Y.ptr[i], nt[i], nt[i], ni[i]}, qT.ptr[i], DMat{Ft.ptr[i], nt[i], nt[i], nt[i]}, qW.ptr[i], qG.ptr[i]});
        ob.sync(s);
        ormqr_vb(ob, false, s);  // Ft = Q_full * blkdiag(L_H, sqrt(s) I) = F^T
        DD_HIP(hipStreamSynchronize(s));
        Y.release();
        qtau.release();
        qT.release();
        qW.release();
        qG.release();
        // Fp[:, j] = F[:, perm(j)] = (row perm(j) of F^T)^T, perm = [nI..nt-1, 0..nI-1]
        Fp.alloc(sf);
        std::vector<double*> srcC(N), srcI(N), dstC(N), dstI(N);
        std::vector<int> actc(N);
        for (int i = 0; i < N; ++i) {
            srcC[i] = Ft.ptr[i] + nI[i];
            srcI[i] = Ft.ptr[i];
            dstC[i] = Fp.ptr[i];
            dstI[i] = Fp.ptr[i] + (int64_t)nc[i] * nt[i];
            actc[i] = nc[i] > 0;
        }
        // dst (nt x nc) = (src rows nI.., all cols)^T : src view is nc x nt with ld nt
        Batch<DMat> sC = mats(srcC, nt, nc, nt, s, &actc), dC = mats(dstC, nt, nt, nc, s, &actc);
        if (sC.size()) copy_vb(sC, dC, true, 1.0, s);
        Batch<DMat> sI = mats(srcI, nt, nI, nt, s), dI = mats(dstI, nt, nt, nI, s);
        copy_vb(sI, dI, true, 1.0, s);
        DD_HIP(hipStreamSynchronize(s));
        Ft.release();
        // the block eigensolver needs S_I = R_II^T R_II with R_II triangular: the QR
        // then factors every column (the trailing n_Ii columns too)
        std::vector<int> nfac(N);
        for (int i = 0; i < N; ++i) nfac[i] = lob ? nt[i] : nc[i];
        Arena ft, fT, fW, fG;
        std::vector<int64_t> a1(N), a2(N), a3(N), a4(N);
        for (int i = 0; i < N; ++i) {
            a1[i] = nt[i];
            a2[i] = qr_t_size(std::max(1, nfac[i]));
            a3[i] = qr_w_size(nt[i]);
            a4[i] = qr_g_size(std::max(1, nfac[i]));
        }
        ft.alloc(a1); fT.alloc(a2); fW.alloc(a3); fG.alloc(a4);
        Batch<QRItem> qb;
        for (int i = 0; i < N; ++i)
            qb.h.push_back(QRItem{DMat{Fp.ptr[i], nt[i], nt[i], nt[i]}, ft.ptr[i], fT.ptr[i], fW.ptr[i], QR_NB, nfac[i], fG.ptr[i]});
        qb.sync(s);
        geqrf_vb(qb, s);
    }
    info.phase_ms[PH_SCHUR] += tm.lap();

    Arena Yev;
    if (lob) {
        eigen_lobpcg(Lv, opt, info, Fp, nc, Yev, s);
    } else {
    // ---- (3.3) reciprocal form: B2 = L_I^{-1} R_II^T, S~ = B2 B2^T, eigenpairs mu < tau --------
    Arena B2, Sm;
    std::vector<int64_t> sI2(N);
    for (int i = 0; i < N; ++i) sI2[i] = (int64_t)nI[i] * nI[i];
    B2.alloc(sI2);
    {
        std::vector<double*> rii(N);
        for (int i = 0; i < N; ++i) rii[i] = Fp.ptr[i] + nc[i] + (int64_t)nc[i] * nt[i];
        Batch<DMat> Rsrc = mats(rii, nt, nI, nI, s);
        Batch<DMat> Bb = mats(B2.ptr, nI, nI, nI, s);
        copy_vb(Rsrc, Bb, true, 1.0, s);  // B2 = G^T, G = (Q^T F_I)[nc:, :] with G^T G = S_I
        DD_HIP(hipStreamSynchronize(s));
        Fp.release();
        Batch<DMat> LI = mats(Lv.L.ptr, ni, nI, nI, s);
        trsm_vb(LI, Bb, false, s);
        Sm.alloc(sI2);
        Batch<GemmItem> g;  // lower triangle of S~ (the tridiagonalisation reads no more)
        for (int i = 0; i < N; ++i)
            g.h.push_back(GemmItem{B2.ptr[i], nI[i], nullptr, 0, Sm.ptr[i], nI[i], nI[i], nI[i], nI[i], 1.0, 0.0});
        g.sync(s);
        syrk_vb(g, s);
        DD_HIP(hipStreamSynchronize(s));
    }
    B2.release();
    Arena td, te, ttau, tpart, tp, tmu;
    std::vector<int64_t> v1(N), vpart(N);
    for (int i = 0; i < N; ++i) { v1[i] = nI[i]; vpart[i] = ceil_div(nI[i], 64) + 1; }
    td.alloc(v1); te.alloc(v1); ttau.alloc(v1); tpart.alloc(vpart); tp.alloc(v1); tmu.alloc(v1);
    {
        Arena tw, taux, typ;
        std::vector<int64_t> sw(N), sa(N, 2 * TRD_NB), syp(N);
        for (int i = 0; i < N; ++i) {
            sw[i] = (int64_t)nI[i] * TRD_NB;
            syp[i] = trd_part_size(nI[i]);
        }
        tw.alloc(sw);
        taux.alloc(sa);
        typ.alloc(syp);
        Batch<TriItem> tb;
        for (int i = 0; i < N; ++i)
            tb.h.push_back(TriItem{DMat{Sm.ptr[i], nI[i], nI[i], nI[i]}, td.ptr[i], te.ptr[i], ttau.ptr[i], tpart.ptr[i],
                                   tp.ptr[i], tw.ptr[i], taux.ptr[i], typ.ptr[i]});
        tb.sync(s);
        sytrd_vb(tb, s);
        DD_HIP(hipStreamSynchronize(s));
    }
    DBuf<int32_t> dcount(N);
    {
        Batch<EigItem> eb;
        for (int i = 0; i < N; ++i) {
            const int cap = (opt.select == DD_SEL_THRESHOLD_CAP) ? std::max(0, opt.nev_cap) : nI[i];
            eb.h.push_back(EigItem{td.ptr[i], te.ptr[i], nI[i], tmu.ptr[i], dcount.p + i, cap, Lv.tau});
        }
        eb.sync(s);
        stebz_vb(eb, s);
    }
    auto hcount = to_host(dcount.p, N, s);
    Lv.p.assign(hcount.begin(), hcount.end());
    Lv.mu.resize(N);
    for (int i = 0; i < N; ++i) {
        Lv.mu[i].resize(Lv.p[i]);
        d2h(Lv.mu[i].data(), tmu.ptr[i], Lv.p[i], s);
    }
    DD_HIP(hipStreamSynchronize(s));
    {
        std::vector<int64_t> sy(N), sw(N);
        for (int i = 0; i < N; ++i) {
            sy[i] = (int64_t)nI[i] * std::max(1, Lv.p[i]);
            sw[i] = stein_work_size(nI[i], Lv.p[i]);
        }
        Yev.alloc(sy);
        Arena wk;
        wk.alloc(sw);
        Batch<VecItem> vb;
        for (int i = 0; i < N; ++i) vb.h.push_back(VecItem{td.ptr[i], te.ptr[i], nI[i], tmu.ptr[i], dcount.p + i, Yev.ptr[i], nI[i], wk.ptr[i]});
        vb.sync(s);
        stein_vb(vb, Lv.mu, 1e-5, s);
        DD_HIP(hipStreamSynchronize(s));
        // back-transform with the tridiagonalisation reflectors (rows 1..nI-1)
        std::vector<int> act(N);
        for (int i = 0; i < N; ++i) act[i] = (Lv.p[i] > 0 && nI[i] > 1);
        Arena oT, oW, oG;
        std::vector<int64_t> s1(N), s2(N), s3(N);
        for (int i = 0; i < N; ++i) {
            s1[i] = qr_t_size(std::max(1, nI[i] - 1));
            s2[i] = qr_w_size(std::max(1, Lv.p[i]));
            s3[i] = qr_g_size(std::max(1, nI[i] - 1));
        }
        oT.alloc(s1); oW.alloc(s2); oG.alloc(s3);
        Batch<ORItem> ob;
        std::vector<double*> taus;
        for (int i = 0; i < N; ++i) {
            if (!act[i]) continue;
            ob.h.push_back(ORItem{DMat{Sm.ptr[i] + 1, nI[i], nI[i] - 1, nI[i] - 1}, oT.ptr[i],
                                  DMat{Yev.ptr[i] + 1, nI[i], nI[i] - 1, Lv.p[i]}, oW.ptr[i], oG.ptr[i]});
            taus.push_back(ttau.ptr[i]);
        }
        if (ob.size()) {
            ob.sync(s);
            build_t_vb(ob, taus, s);
            ormqr_vb(ob, false, s);
        }
        DD_HIP(hipStreamSynchronize(s));
    }
    Sm.release();
    }
    info.phase_ms[PH_EIG] += tm.lap();

    // ---- Z_i = orth(L_I^{-T} Y_keep)  (D_i u with Boolean D_i) --------------------------------
    {
        std::vector<int64_t> sz(N);
        std::vector<int> act(N);
        for (int i = 0; i < N; ++i) { sz[i] = (int64_t)nI[i] * Lv.p[i]; act[i] = Lv.p[i] > 0; }
        Lv.Z.alloc(sz);
        std::vector<int>& pp = Lv.p;
        Batch<DMat> LI = mats(Lv.L.ptr, ni, nI, nI, s, &act);
        Batch<DMat> Yb = mats(Yev.ptr, nI, nI, pp, s, &act);
        if (Yb.size()) {
            trsm_vb(LI, Yb, true, s);
            Arena zt, zT, zW, zG;
            std::vector<int64_t> a1(N), a2(N), a3(N), a4(N);
            for (int i = 0; i < N; ++i) {
                a1[i] = std::max(1, pp[i]);
                a2[i] = qr_t_size(std::max(1, pp[i]));
                a3[i] = qr_w_size(std::max(1, pp[i]));
                a4[i] = qr_g_size(std::max(1, pp[i]));
            }
            zt.alloc(a1); zT.alloc(a2); zW.alloc(a3); zG.alloc(a4);
            Batch<QRItem> qb;
            Batch<ORItem> ob;
            for (int i = 0; i < N; ++i) {
                if (!act[i]) continue;
                qb.h.push_back(QRItem{DMat{Yev.ptr[i], nI[i], nI[i], pp[i]}, zt.ptr[i], zT.ptr[i], zW.ptr[i], QR_NB, pp[i], zG.ptr[i]});
                ob.h.push_back(ORItem{DMat{Yev.ptr[i], nI[i], nI[i], pp[i]}, zT.ptr[i], DMat{Lv.Z.ptr[i], nI[i], nI[i], pp[i]}, zW.ptr[i], zG.ptr[i]});
            }
            qb.sync(s);
            ob.sync(s);
            geqrf_vb(qb, s);
            Batch<DMat> Zb = mats(Lv.Z.ptr, nI, nI, pp, s, &act);
            set_identity_vb(Zb, 1.0, s);
            orgqr_vb(ob, s);
            DD_HIP(hipStreamSynchronize(s));
        }
    }
    Yev.release();
    info.phase_ms[PH_BASIS] += tm.lap();

    // ---- W_i = L_i^{-1}: the local solves of the apply become two triangular
    // matrix-vector products (HBM-bound, fully parallel); in the FP32 form only
    // the subdomains that fell back need it (the others have W_i in FP32) ------
    const std::vector<int>& fp64 = Lv.fp64;
    Lv.L32.release();
    Lv.jd.release();
    {
        std::vector<int64_t> sa(N);
        for (int i = 0; i < N; ++i) sa[i] = fp64[i] ? (int64_t)ni[i] * ni[i] : 1;
        Lv.W.alloc(sa);
        Batch<DMat> Wb = mats(Lv.W.ptr, ni, ni, ni, s, &fp64);
        if (Wb.size()) {
            set_identity_vb(Wb, 1.0, s);
            Batch<DMat> Lb = mats(Lv.L.ptr, ni, ni, ni, s, &fp64);
            trsm_vb(Lb, Wb, false, s, true);
        }
        DD_HIP(hipStreamSynchronize(s));
        Lv.L.release();
    }
    info.phase_ms[PH_CHOL] += tm.lap();

    // ---- coarse operator E = Z^T A Z (block (i,j) from the rows of Omega_j owned by i) ----------
    Lv.pcnt = upload(std::vector<int32_t>(Lv.p.begin(), Lv.p.end()), s);
    Lv.hoffC.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) Lv.hoffC[i + 1] = Lv.hoffC[i] + Lv.p[i];
    Lv.offC = upload(Lv.hoffC, s);
    Lv.nC = Lv.hoffC[N];
    Lv.dZ.alloc(N);
    h2d(Lv.dZ.p, Lv.Z.ptr.data(), N, s);
    DD_HIP(hipStreamSynchronize(s));
    const int64_t nC = Lv.nC;
    if (nC > 0) {
        SubInfo S = Lv.sub();
        // block graph of E and the symbolic block Cholesky
        {
            DBuf<uint8_t> adj((size_t)N * N);
            DD_HIP(hipMemsetAsync(adj.p, 0, adj.bytes(), s));
            block_adjacency(A, Lv.part.p, N, adj.p, s);
            Lv.hadj = to_host(adj.p, (size_t)N * N, s);
            Lv.E.symbolic(Lv.hadj, Lv.p, Lv.hoffC);
            Lv.E.allocate(s);
        }
        DBuf<int32_t> cnt((size_t)N * N);
        DD_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes(), s));
        pair_counts(S, cnt.p, s);
        auto hc = to_host(cnt.p, (size_t)N * N, s);
        std::vector<int64_t> pairoff((size_t)N * N, 0);
        std::vector<PairItem> pairs, dense_pairs;
        const bool keep_dense = nC <= 4096;
        DBuf<double> Ed;
        if (keep_dense) {
            Ed.alloc((size_t)nC * nC);
            fill(Ed.p, Ed.n, 0.0, s);
        }
        int64_t pos = 0;
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const int64_t key = (int64_t)j * N + i;
                pairoff[key] = pos;
                if (hc[key] > 0) {
                    if (Lv.p[i] > 0 && Lv.p[j] > 0) {
                        int ld = 0;
                        double* out = (Lv.E.pos[i] >= Lv.E.pos[j]) ? Lv.E.block(i, j, &ld) : nullptr;
                        if (out) pairs.push_back(PairItem{i, j, hc[key], pos, out, ld});
                        if (keep_dense && (i == j || out || Lv.E.block(j, i, &ld)))
                            dense_pairs.push_back(PairItem{i, j, hc[key], pos, Ed.p + Lv.hoffC[i] + Lv.hoffC[j] * nC, nC});
                    }
                    pos += hc[key];
                }
            }
        DBuf<int64_t> dpo = upload(pairoff, s);
        DBuf<int32_t> cursor((size_t)N * N), zr(pos), pr(pos);
        DD_HIP(hipMemsetAsync(cursor.p, 0, cursor.bytes(), s));
        pair_fill(S, dpo.p, cursor.p, zr.p, pr.p, s);
        Arena P;
        std::vector<int64_t> sp(N);
        for (int j = 0; j < N; ++j) sp[j] = (int64_t)ni[j] * Lv.p[j];
        P.alloc(sp);
        DBuf<double*> dP(N);
        h2d(dP.p, P.ptr.data(), N, s);
        build_p(A, S, dP.p, ni, Lv.p, s);
        DBuf<PairItem> dpairs = upload(pairs, s);
        assemble_e(S, dpairs.p, pairs, Lv.p, dP.p, zr.p, pr.p, s);
        if (keep_dense) {
            DBuf<PairItem> dd2 = upload(dense_pairs, s);
            assemble_e(S, dd2.p, dense_pairs, Lv.p, dP.p, zr.p, pr.p, s);
            Lv.Ecopy = to_host(Ed.p, (size_t)nC * nC, s);
        }
        DD_HIP(hipStreamSynchronize(s));
        if (next) build_e_csr(Lv, *next, s);
        info.phase_ms[PH_E] += tm.lap();
        if (!next) {
            const int bad = Lv.E.factor(s);
            DD_CHECK(bad == 0, DD_ERR_NOT_SPD, "coarse operator E is not positive definite");
            info.phase_ms[PH_EFACT] += tm.lap();
        }
    }

    // ---- apply workspace ----
    Lv.rloc.alloc(std::max<int64_t>(1, Lv.hoffO[N]));
    Lv.yC.alloc(std::max<int64_t>(1, nC));
    {
        std::vector<int64_t> poff(N + 1, 0);
        for (int i = 0; i < N; ++i) poff[i + 1] = poff[i] + trmv_part_size(ni[i]);
        Lv.yloc.alloc(std::max<int64_t>(1, Lv.hoffO[N]));
        Lv.tpart.alloc(std::max<int64_t>(1, poff[N]));
        Lv.Tb.h.clear();
        Lv.Tb32.h.clear();
        for (int i = 0; i < N; ++i) {
            if (!fp64[i])
                Lv.Tb32.h.push_back(TrmvItem32{Lv.W32.ptr[i], ni[i], ni[i], Lv.rloc.p + Lv.hoffO[i],
                                               Lv.yloc.p + Lv.hoffO[i], Lv.tpart.p + poff[i]});
            else
                Lv.Tb.h.push_back(TrmvItem{Lv.W.ptr[i], ni[i], ni[i], Lv.rloc.p + Lv.hoffO[i], Lv.yloc.p + Lv.hoffO[i],
                                           Lv.tpart.p + poff[i]});
        }
        if (!Lv.Tb32.h.empty()) Lv.Tb32.sync(s);
        if (!Lv.Tb.h.empty()) Lv.Tb.sync(s);
        if (Lv.Tb32.h.empty()) Lv.W32.release();
        if (Lv.Tb.h.empty()) Lv.W.release();
    }
    info.phase_ms[PH_OTHER] += tm.lap();
}

// ---------------------------------------------------------------------------
// multilevel recursion (multilevel remark of Sec. 3.2): E of one level becomes
// the CSR matrix of the next
// ---------------------------------------------------------------------------
struct EcsrItem {
    const double* src;  // dense block of E inside a factor panel
    int ld;
    int trans;          // 0: element (a, b) at src[a + b ld]; 1: at src[b + a ld]; 2: lower triangle mirrored
    int pi, pj;
    int64_t row0;       // coarse index of the block's first row
    int64_t coloff;     // offset of the block's first column within each CSR row
    int64_t col0;       // coarse index of the block's first column
};
struct OpEcsr {
    const EcsrItem* it;
    const int32_t* rowptr;
    int32_t* colind;
    double* val;
    __device__ int tiles(int q) const { return ((it[q].pi + 63) / 64) * ((it[q].pj + 63) / 64); }
    __device__ void operator()(int q, int t) const {
        const EcsrItem& I = it[q];
        const int tm = (I.pi + 63) / 64;
        const int a0 = (t % tm) * 64, b0 = (t / tm) * 64;
        for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
            const int a = a0 + e / 64, b = b0 + e % 64;
            if (a >= I.pi || b >= I.pj) continue;
            const int64_t dst = rowptr[I.row0 + a] + I.coloff + b;
            colind[dst] = (int32_t)(I.col0 + b);
            int r = a, c = b;
            if (I.trans == 1 || (I.trans == 2 && b > a)) { r = b; c = a; }  // 2: diagonal block, lower mirrored
            val[dst] = I.src[r + (int64_t)c * I.ld];
        }
    }
};

// E (assembled in the factor panels, not yet factored) -> CSR of `next`:
// full symmetric storage, row r of block i holds the blocks j in {i} U
// neighbours(i) with p_j > 0, in increasing j (so columns are sorted).
static void build_e_csr(Level& Lv, Level& next, hipStream_t s) {
    const int N = Lv.N;
    const auto& P = Lv.p;
    std::vector<std::vector<int>> nb(N);
    std::vector<int64_t> rowlen(N, 0);
    for (int i = 0; i < N; ++i) {
        if (P[i] <= 0) continue;
        for (int j = 0; j < N; ++j)
            if (P[j] > 0 && (j == i || Lv.hadj[(size_t)i * N + j])) {
                nb[i].push_back(j);
                rowlen[i] += P[j];
            }
    }
    const int64_t nC = Lv.nC;
    std::vector<int32_t> rp(nC + 1, 0);
    int64_t nnz = 0;
    for (int i = 0; i < N; ++i)
        for (int a = 0; a < P[i]; ++a) {
            rp[Lv.hoffC[i] + a] = (int32_t)nnz;
            nnz += rowlen[i];
            DD_CHECK(nnz < INT32_MAX, DD_ERR_INVALID_ARG, "coarse operator too large for a 32-bit CSR (use the nev cap)");
        }
    rp[nC] = (int32_t)nnz;
    std::vector<EcsrItem> items;
    for (int i = 0; i < N; ++i) {
        int64_t off = 0;
        for (int j : nb[i]) {
            int ld = 0;
            EcsrItem e{};
            if (i == j) {
                e.src = Lv.E.block(i, i, &ld);
                e.trans = 2;
            } else if (Lv.E.pos[i] >= Lv.E.pos[j]) {
                e.src = Lv.E.block(i, j, &ld);
                e.trans = 0;
            } else {
                e.src = Lv.E.block(j, i, &ld);
                e.trans = 1;
            }
            DD_CHECK(e.src != nullptr, DD_ERR_INTERNAL, "coarse block missing from the factor structure");
            e.ld = ld;
            e.pi = P[i];
            e.pj = P[j];
            e.row0 = Lv.hoffC[i];
            e.coloff = off;
            e.col0 = Lv.hoffC[j];
            items.push_back(e);
            off += P[j];
        }
    }
    next.n = nC;
    next.nnz = nnz;
    next.rowptr = upload(rp, s);
    next.colind.alloc(nnz);
    next.val.alloc(nnz);
    DBuf<EcsrItem> dit = upload(items, s);
    int64_t tiles = 0;
    for (auto& e : items) tiles += (int64_t)ceil_div(e.pi, 64) * ceil_div(e.pj, 64);
    launch_tiles(OpEcsr{dit.p, next.rowptr.p, next.colind.p, next.val.p}, (int)items.size(), tiles, s, "e_csr");
    DD_HIP(hipStreamSynchronize(s));
}

// Partition of the next level (R8): the nodes of E's block graph are this
// level's subdomains; seeded greedy graph growing into ceil(N / coarsen) parts
// (seed 0), expanded to the coarse dofs, empty parts removed.
static void partition_next_batch(const Level& Lv, Level& next, int coarsen, hipStream_t s);

static void partition_next(const Level& Lv, Level& next, int coarsen, hipStream_t s) {
    if (!Lv.hsub.empty()) {
        partition_next_batch(Lv, next, coarsen, s);
        return;
    }
    const int N = Lv.N;
    std::vector<int32_t> rp(N + 1, 0), ci;
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j)
            if (j != i && Lv.hadj[(size_t)i * N + j]) ci.push_back(j);
        rp[i + 1] = (int32_t)ci.size();
    }
    if (ci.empty()) ci.push_back(0);  // keeps the device arrays non-empty; rp says no edges
    const int N2 = std::min(N, ceil_div(N, std::max(1, coarsen)));
    DBuf<int32_t> drp = upload(rp, s), dci = upload(ci, s);
    DBuf<double> dval(std::max<size_t>(1, ci.size()));
    CsrDev G{N, (int64_t)rp[N], drp.p, dci.p, dval.p};
    DBuf<int32_t> dpart(N);
    ggg_partition(G, N2, 0, dpart.p, s);
    std::vector<int32_t> pb = to_host(dpart.p, N, s);
    std::vector<int32_t> used(N2, 0);
    for (int i = 0; i < N; ++i)
        if (Lv.p[i] > 0) used[pb[i]] = 1;
    std::vector<int32_t> remap(N2, -1);
    int cnt = 0;
    for (int k = 0; k < N2; ++k)
        if (used[k]) remap[k] = cnt++;
    std::vector<int32_t> part2(Lv.nC);
    for (int i = 0; i < N; ++i)
        for (int a = 0; a < Lv.p[i]; ++a) part2[Lv.hoffC[i] + a] = remap[pb[i]];
    next.part = upload(part2, s);
    next.N = cnt;
    next.delta = Lv.delta;
    next.tau = Lv.tau;
    DD_HIP(hipStreamSynchronize(s));
}

// The same partition of a batch level, system by system: the subdomain graph
// of each system gets its own ceil(N_j / coarsen) parts by the same rule and
// seed, so every system's next level is the one its own setup would build;
// the parts, coarse dofs and their system ranges stay contiguous per system.
static void partition_next_batch(const Level& Lv, Level& next, int coarsen, hipStream_t s) {
    const int N = Lv.N, ns = (int)Lv.hsub.size() - 1;
    std::vector<int32_t> part2(Lv.nC);
    next.hsub.assign(1, 0);
    next.hseg.assign(1, 0);
    int total = 0;
    for (int j = 0; j < ns; ++j) {
        const int s0 = Lv.hsub[j], s1 = Lv.hsub[j + 1], Nj = s1 - s0;
        if (Nj == 0) {  // this system kept no coarse mode on the level above: nothing to partition
            next.hsub.push_back(total);
            next.hseg.push_back(Lv.hoffC[s1]);
            continue;
        }
        std::vector<int32_t> rp(Nj + 1, 0), ci;
        for (int i = 0; i < Nj; ++i) {
            for (int k = 0; k < Nj; ++k)
                if (k != i && Lv.hadj[(size_t)(s0 + i) * N + (s0 + k)]) ci.push_back(k);
            rp[i + 1] = (int32_t)ci.size();
        }
        if (ci.empty()) ci.push_back(0);
        const int N2 = std::max(1, std::min(Nj, ceil_div(Nj, std::max(1, coarsen))));
        DBuf<int32_t> drp = upload(rp, s), dci = upload(ci, s);
        DBuf<double> dval(std::max<size_t>(1, ci.size()));
        CsrDev G{Nj, (int64_t)rp[Nj], drp.p, dci.p, dval.p};
        DBuf<int32_t> dpart(std::max(1, Nj));
        ggg_partition(G, N2, 0, dpart.p, s);
        std::vector<int32_t> pb = to_host(dpart.p, Nj, s);
        std::vector<int32_t> used(N2, 0), remap(N2, -1);
        for (int i = 0; i < Nj; ++i)
            if (Lv.p[s0 + i] > 0) used[pb[i]] = 1;
        int cnt = 0;
        for (int k = 0; k < N2; ++k)
            if (used[k]) remap[k] = cnt++;
        for (int i = 0; i < Nj; ++i)
            for (int a = 0; a < Lv.p[s0 + i]; ++a) part2[Lv.hoffC[s0 + i] + a] = total + remap[pb[i]];
        total += cnt;
        next.hsub.push_back(total);
        next.hseg.push_back(Lv.hoffC[s1]);
    }
    std::vector<int32_t> sid(std::max<int64_t>(1, Lv.nC), 0);
    for (int j = 0; j < ns; ++j)
        for (int64_t d = next.hseg[j]; d < next.hseg[j + 1]; ++d) sid[d] = j;
    next.part = upload(part2, s);
    next.dseg = upload(next.hseg, s);
    next.seg_id = upload(sid, s);
    next.N = total;
    next.delta = Lv.delta;
    next.tau = Lv.tau;
    DD_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// apply and Krylov solvers
// ---------------------------------------------------------------------------
__global__ void k_axpy2(double* x, double* r, const double* p, const double* q, double alpha, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        r[i] -= alpha * q[i];
    }
}
__global__ void k_xpby(const double* z, double* p, double beta, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}
__global__ void k_sub(const double* b, double* r, int64_t n) {  // r = b - r
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        r[i] = b[i] - r[i];
}
__global__ void k_diff(const double* a, const double* b, double* c, int64_t n) {  // c = a - b
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c[i] = a[i] - b[i];
}
static int vgrid(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

static double dot_host(Handle& H, const double* x, const double* y, int64_t n, hipStream_t s) {
    dot(x, y, n, 1, H.partial.p, H.dots.p, s);
    DD_HIP(hipMemcpyAsync(H.hpin, H.dots.p, sizeof(double), hipMemcpyDeviceToHost, s));
    DD_HIP(hipStreamSynchronize(s));
    return H.hpin[0];
}

constexpr double kInnerRtol = 1e-4;  // coarse solves by PCG on levels >= 2 (Sec. 4)

static int krylov(Handle& H, size_t m, const double* b, double* x, double rtol, int maxit, bool flexible,
                  bool true_res, int* iters, double* relres, hipStream_t s);
static int gmres(Handle& H, size_t m, const double* b, double* x, double rtol, int maxit, int restart, int* iters,
                 double* relres, hipStream_t s);
static int krylov_seg(Handle& H, size_t m, const double* b, double* x, double rtol, int maxit, bool flexible,
                      bool true_res, int* iters, double* relres, hipStream_t s);

// y := E_m^{-1} y: exact block Cholesky solve on the last level, otherwise PCG
// (deflated variant: right-preconditioned GMRES(30)) on E_m, the next level's
// matrix, to kInnerRtol, preconditioned by the next level, from x0 = 0.
static void coarse_solve(Handle& H, size_t m, double* y, hipStream_t s) {
    Level& Lv = *H.lv[m];
    if (m + 1 >= H.lv.size()) {
        Lv.E.solve(y, s);
        return;
    }
    Level& Nx = *H.lv[m + 1];
    int its = 0;
    double rr = 0.0;
    fill(Nx.kx.p, Nx.n, 0.0, s);
    // a batch solves each system's coarse system on its own (the systems' inner
    // levels are kept apart by the per-system partition of every level)
    const int rc = H.opt.schwarz == DD_SCHWARZ_DEFLATED
                       ? gmres(H, m + 1, y, Nx.kx.p, kInnerRtol, 1000, 30, &its, &rr, s)
                   : H.nsys() > 1
                       ? krylov_seg(H, m + 1, y, Nx.kx.p, kInnerRtol, 1000, false, false, nullptr, nullptr, s)
                       : krylov(H, m + 1, y, Nx.kx.p, kInnerRtol, 1000, false, false, &its, &rr, s);
    DD_CHECK(rc >= 0, rc, "inner coarse solve failed");
    DD_HIP(hipMemcpyAsync(y, Nx.kx.p, Nx.n * sizeof(double), hipMemcpyDeviceToDevice, s));
}

// z[g] = base[g] + (local solution of g's own part at g): the prolongation of
// the restricted method with the Boolean partition of unity (base optional)
__global__ void k_ras_prolong(const double* rloc, const int64_t* offO, const int32_t* part, const int32_t* ilocal,
                              const double* base, double* z, int64_t n) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        const double v = rloc[offO[part[g]] + ilocal[g]];
        z[g] = base ? base[g] + v : v;
    }
}

// rloc_i := W_i^T W_i rloc_i for every subdomain (FP32 and FP64 inverses in
// their own launches; each writes only its subdomains' segments)
static void local_solves(Level& Lv, hipStream_t s) {
    if (!Lv.Tb32.h.empty()) trinv_apply_vb(Lv.Tb32, s);
    if (!Lv.Tb.h.empty()) trinv_apply_vb(Lv.Tb, s);
}

// z = M_deflated r = y + M_RAS (r - A y), y = Z E^{-1} Z^T r (Sec. 4): the
// coarse correction first, then the restricted one-level method on the
// residual it leaves.  The coarse solve of a level that is not the last is
// right-preconditioned GMRES(30) to kInnerRtol with the next level's M_deflated.
static void apply_deflated(Handle& H, size_t m, const double* r, double* z, hipStream_t s) {
    Level& Lv = *H.lv[m];
    const int64_t n = Lv.n;
    const double* rr = r;
    const double* base = nullptr;
    if (Lv.nC > 0) {
        SubInfo S = Lv.sub();
        restrict_coarse(S, Lv.nC, r, Lv.yC.p, s);
        coarse_solve(H, m, Lv.yC.p, s);
        fill(Lv.dy.p, n, 0.0, s);
        prolong_coarse(S, Lv.offI.p, Lv.hoffI[Lv.N], Lv.yC.p, Lv.dy.p, s);
        spmv(Lv.A(), Lv.dy.p, Lv.dt.p, 1, s);
        hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, r, Lv.dt.p, n);  // dt = r - A y
        rr = Lv.dt.p;
        base = Lv.dy.p;
    }
    gather(rr, Lv.omega_flat.p, Lv.hoffO[Lv.N], Lv.rloc.p, s);
    local_solves(Lv, s);
    hipLaunchKernelGGL(k_ras_prolong, dim3(vgrid(n)), dim3(256), 0, s, Lv.rloc.p, Lv.offO.p, Lv.part.p, Lv.ilocal.p,
                       base, z, n);
    launch_check("apply_deflated");
}

// z = M_m^{-1} r: the additive preconditioner (2.1) of level m, or the
// deflated one of Sec. 4
static void apply_level(Handle& H, size_t m, const double* r, double* z, hipStream_t s) {
    if (H.opt.schwarz == DD_SCHWARZ_DEFLATED) {
        apply_deflated(H, m, r, z, s);
        return;
    }
    Level& Lv = *H.lv[m];
    gather(r, Lv.omega_flat.p, Lv.hoffO[Lv.N], Lv.rloc.p, s);
    local_solves(Lv, s);  // rloc_i := W_i^T W_i rloc_i = A_ii^{-1} rloc_i
    scatter_sum(Lv.rloc.p, Lv.memb_ptr.p, Lv.memb.p, Lv.n, z, false, s);
    if (Lv.nC > 0) {
        SubInfo S = Lv.sub();
        restrict_coarse(S, Lv.nC, r, Lv.yC.p, s);
        coarse_solve(H, m, Lv.yC.p, s);
        prolong_coarse(S, Lv.offI.p, Lv.hoffI[Lv.N], Lv.yC.p, z, s);
    }
}

static void alloc_krylov(Level& Lv, bool deflated) {
    const int64_t n = std::max<int64_t>(1, Lv.n);
    if (deflated) {
        Lv.dy.alloc(n);
        Lv.dt.alloc(n);
    }
    Lv.kr.alloc(n);
    Lv.kz.alloc(n);
    Lv.kp.alloc(n);
    Lv.kq.alloc(n);
    Lv.kro.alloc(n);
    Lv.kx.alloc(n);
}

// PCG (R6) on the matrix of level m with the preconditioner of level m; x
// holds x0 on entry.  Stop when the recurrence residual satisfies
// ||r_k|| <= rtol ||b||.  flexible: Polak-Ribiere beta for a preconditioner
// that varies between iterations (inner solves on lower levels, R8).
static int krylov(Handle& H, size_t m, const double* b, double* x, double rtol, int maxit, bool flexible,
                  bool true_res, int* iters, double* relres, hipStream_t s) {
    Level& Lv = *H.lv[m];
    const int64_t n = Lv.n;
    const CsrDev A = Lv.A();
    double *r = Lv.kr.p, *z = Lv.kz.p, *p = Lv.kp.p, *q = Lv.kq.p, *ro = Lv.kro.p;
    const double bn = std::sqrt(dot_host(H, b, b, n, s));
    DD_CHECK(std::isfinite(bn), DD_ERR_NAN, "right-hand side contains NaN/Inf");
    if (bn == 0.0) {
        fill(x, n, 0.0, s);
        *iters = 0;
        *relres = 0.0;
        return DD_OK;
    }
    spmv(A, x, r, 1, s);
    hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b, r, n);
    double rn = std::sqrt(dot_host(H, r, r, n, s));
    int its = 0;
    bool conv = rn <= rtol * bn;
    if (!conv) {
        apply_level(H, m, r, z, s);
        DD_HIP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        double rz = dot_host(H, r, z, n, s);
        for (its = 1; its <= maxit; ++its) {
            spmv(A, p, q, 1, s);
            const double pq = dot_host(H, p, q, n, s);
            DD_CHECK(std::isfinite(pq), DD_ERR_NAN, "PCG produced NaN");
            const double alpha = rz / pq;
            if (flexible) DD_HIP(hipMemcpyAsync(ro, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_axpy2, dim3(vgrid(n)), dim3(256), 0, s, x, r, p, q, alpha, n);
            rn = std::sqrt(dot_host(H, r, r, n, s));
            if (rn <= rtol * bn) { conv = true; break; }
            apply_level(H, m, r, z, s);
            double beta;
            if (flexible) {
                hipLaunchKernelGGL(k_diff, dim3(vgrid(n)), dim3(256), 0, s, r, ro, q, n);  // q := r - r_old
                beta = dot_host(H, z, q, n, s) / rz;
                rz = dot_host(H, r, z, n, s);
            } else {
                const double rzn = dot_host(H, r, z, n, s);
                beta = rzn / rz;
                rz = rzn;
            }
            hipLaunchKernelGGL(k_xpby, dim3(vgrid(n)), dim3(256), 0, s, z, p, beta, n);
        }
        if (its > maxit) its = maxit;
    }
    double rel = rn / bn;
    if (true_res) {
        spmv(A, x, r, 1, s);
        hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b, r, n);
        rel = std::sqrt(dot_host(H, r, r, n, s)) / bn;
        DD_CHECK(std::isfinite(rel), DD_ERR_NAN, "PCG produced NaN");
    }
    *iters = its;
    *relres = rel;
    return conv ? DD_OK : DD_WARN_MAXIT;
}

// ---------------------------------------------------------------------------
// PCG as a captured graph (the host-driven krylov() above, with its scalars on
// the device).  One iteration: q = A p; pq = p.q; alpha = rz / pq; x += alpha p,
// r -= alpha q; rn2 = r.r; stop test sqrt(rn2) <= rtol ||b|| (or maxit); z = M r;
// rzn = r.z; beta = rzn / rz, rz = rzn; p = z + beta p.  After the stop every
// update is skipped (state != 0), so the iterate stays that of the step that
// stopped, and the iterations replayed past it only cost time.  The divisions
// and dots are the host loop's (IEEE double, the same deterministic dot
// kernels), so the iterates agree bit for bit.
// state: 0 running, 1 converged, 2 maxit, 3 non-finite p.q
// ---------------------------------------------------------------------------
__global__ void k_g_alpha(double* S) {
    if (S[G_STATE] != 0.0) {
        S[G_ALPHA] = 0.0;
        return;
    }
    if (!isfinite(S[G_PQ])) {
        S[G_STATE] = 3.0;
        S[G_ALPHA] = 0.0;
        return;
    }
    S[G_ALPHA] = S[G_RZ] / S[G_PQ];
}
__global__ void k_g_check(double* S) {
    if (S[G_STATE] != 0.0) return;
    S[G_ITS] += 1.0;
    if (sqrt(S[G_RN2]) <= S[G_THR]) S[G_STATE] = 1.0;
    else if (S[G_ITS] >= S[G_MAXIT]) S[G_STATE] = 2.0;
}
__global__ void k_g_beta(double* S) {
    if (S[G_STATE] != 0.0) return;
    S[G_BETA] = S[G_RZN] / S[G_RZ];
    S[G_RZ] = S[G_RZN];
}
__global__ void k_g_axpy2(double* x, double* r, const double* p, const double* q, const double* S, int64_t n) {
    const double a = S[G_ALPHA];
    if (a == 0.0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += a * p[i];
        r[i] -= a * q[i];
    }
}
__global__ void k_g_xpby(const double* z, double* p, const double* S, int64_t n) {
    if (S[G_STATE] != 0.0) return;
    const double b = S[G_BETA];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + b * p[i];
}

static void graph_iteration(Handle& H, double* S, hipStream_t s) {
    Level& Lv = *H.lv[0];
    const int64_t n = Lv.n;
    const CsrDev A = Lv.A();
    double *x = Lv.kx.p, *r = Lv.kr.p, *z = Lv.kz.p, *p = Lv.kp.p, *q = Lv.kq.p;
    spmv(A, p, q, 1, s);
    dot(p, q, n, 1, H.partial.p, S + G_PQ, s);
    hipLaunchKernelGGL(k_g_alpha, dim3(1), dim3(1), 0, s, S);
    hipLaunchKernelGGL(k_g_axpy2, dim3(vgrid(n)), dim3(256), 0, s, x, r, p, q, S, n);
    dot(r, r, n, 1, H.partial.p, S + G_RN2, s);
    hipLaunchKernelGGL(k_g_check, dim3(1), dim3(1), 0, s, S);
    apply_level(H, 0, r, z, s);
    dot(r, z, n, 1, H.partial.p, S + G_RZN, s);
    hipLaunchKernelGGL(k_g_beta, dim3(1), dim3(1), 0, s, S);
    hipLaunchKernelGGL(k_g_xpby, dim3(vgrid(n)), dim3(256), 0, s, z, p, S, n);
    launch_check("graph_pcg");
}

static int krylov_graph(Handle& H, const double* b, double* xio, double rtol, int maxit, int* iters, double* relres,
                        hipStream_t s) {
    Level& Lv = *H.lv[0];
    const int64_t n = Lv.n;
    const CsrDev A = Lv.A();
    if (!H.gp || H.gp->chunk != H.opt.graph_pcg) {
        H.gp = std::make_unique<GraphPcg>();
        GraphPcg& G = *H.gp;
        G.chunk = H.opt.graph_pcg;
        G.S.alloc(G_NSLOT);
        DD_HIP(hipHostMalloc(&G.hS, G_NSLOT * sizeof(double)));
        DD_HIP(hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking));
        DD_HIP(hipStreamBeginCapture(G.cs, hipStreamCaptureModeThreadLocal));
        try {
            graph_iteration(H, G.S.p, G.cs);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(G.cs, &g);
            if (g) (void)hipGraphDestroy(g);
            H.gp.reset();
            throw;
        }
        DD_HIP(hipStreamEndCapture(G.cs, &G.graph));
        DD_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
    }
    GraphPcg& G = *H.gp;
    double *x = Lv.kx.p, *r = Lv.kr.p, *z = Lv.kz.p, *p = Lv.kp.p;
    DD_HIP(hipMemcpyAsync(x, xio, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    // the start as in krylov(): r = b - A x, stop test, z = M r, p = z, rz = r.z
    const double bn = std::sqrt(dot_host(H, b, b, n, s));
    DD_CHECK(std::isfinite(bn), DD_ERR_NAN, "right-hand side contains NaN/Inf");
    if (bn == 0.0) {
        fill(xio, n, 0.0, s);
        *iters = 0;
        *relres = 0.0;
        return DD_OK;
    }
    spmv(A, x, r, 1, s);
    hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b, r, n);
    double rn = std::sqrt(dot_host(H, r, r, n, s));
    int its = 0;
    bool conv = rn <= rtol * bn;
    if (!conv && maxit > 0) {
        apply_level(H, 0, r, z, s);
        DD_HIP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        const double rz = dot_host(H, r, z, n, s);
        double* hS = G.hS;
        for (int k = 0; k < G_NSLOT; ++k) hS[k] = 0.0;
        hS[G_RZ] = rz;
        hS[G_THR] = rtol * bn;
        hS[G_MAXIT] = maxit;
        h2d(G.S.p, hS, G_NSLOT, s);
        // batches of replays between host checks, sized from the observed residual
        // contraction so that few iterations run past the stop (those only cost time)
        int batch = std::min(2, G.chunk);
        double rprev = rn;
        for (;;) {
            for (int j = 0; j < batch; ++j) DD_HIP(hipGraphLaunch(G.exec, s));
            d2h(hS, G.S.p, G_NSLOT, s);
            DD_HIP(hipStreamSynchronize(s));
            if (hS[G_STATE] != 0.0) break;
            const double rcur = std::sqrt(hS[G_RN2]);
            const double rate = std::pow(rcur / rprev, 1.0 / batch);
            rprev = rcur;
            double est = G.chunk;
            if (rate > 0.0 && rate < 1.0) est = std::log(hS[G_THR] / rcur) / std::log(rate);
            batch = (int)std::max(1.0, std::min<double>(G.chunk, std::floor(est)));
        }
        DD_CHECK(hS[G_STATE] != 3.0, DD_ERR_NAN, "PCG produced NaN");
        its = (int)hS[G_ITS];
        conv = hS[G_STATE] == 1.0;
    }
    // true residual at exit
    spmv(A, x, r, 1, s);
    hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b, r, n);
    const double rel = std::sqrt(dot_host(H, r, r, n, s)) / bn;
    DD_CHECK(std::isfinite(rel), DD_ERR_NAN, "PCG produced NaN");
    DD_HIP(hipMemcpyAsync(xio, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    *iters = its;
    *relres = rel;
    return conv ? DD_OK : DD_WARN_MAXIT;
}

// ---------------------------------------------------------------------------
// Several right-hand sides in lockstep (two levels, additive, one system):
// every column runs the host loop of krylov() with its scalars on the device
// (as in the graph iteration), while the SpMV reads A and the local solves read
// every W_i once per group of up to kMrhs columns.  Each column's arithmetic is
// that of a single right-hand side, so every column equals its own dd_pcg call
// bit for bit; a column that has stopped keeps its iterate (alpha = 0, no p
// update) while the others go on.
// ---------------------------------------------------------------------------
__global__ void k_b_alpha(double* S, int K) {
    const int k = threadIdx.x;
    if (k >= K) return;
    double* a = S + G_ALPHA * kMrhs + k;
    if (S[G_STATE * kMrhs + k] != 0.0) {
        *a = 0.0;
        return;
    }
    const double pq = S[G_PQ * kMrhs + k];
    if (!isfinite(pq)) {
        S[G_STATE * kMrhs + k] = 3.0;
        *a = 0.0;
        return;
    }
    *a = S[G_RZ * kMrhs + k] / pq;
}
__global__ void k_b_check(double* S, int K) {
    const int k = threadIdx.x;
    if (k >= K || S[G_STATE * kMrhs + k] != 0.0) return;
    S[G_ITS * kMrhs + k] += 1.0;
    if (sqrt(S[G_RN2 * kMrhs + k]) <= S[G_THR * kMrhs + k]) S[G_STATE * kMrhs + k] = 1.0;
    else if (S[G_ITS * kMrhs + k] >= S[G_MAXIT * kMrhs + k]) S[G_STATE * kMrhs + k] = 2.0;
}
__global__ void k_b_beta(double* S, int K) {
    const int k = threadIdx.x;
    if (k >= K || S[G_STATE * kMrhs + k] != 0.0) return;
    S[G_BETA * kMrhs + k] = S[G_RZN * kMrhs + k] / S[G_RZ * kMrhs + k];
    S[G_RZ * kMrhs + k] = S[G_RZN * kMrhs + k];
}
// column k = blockIdx.y
__global__ void k_b_axpy2(double* x, double* r, const double* p, const double* q, const double* S, int64_t n) {
    const int k = blockIdx.y;
    const double a = S[G_ALPHA * kMrhs + k];
    if (a == 0.0) return;
    double *xk = x + k * n, *rk = r + k * n;
    const double *pk = p + k * n, *qk = q + k * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        xk[i] += a * pk[i];
        rk[i] -= a * qk[i];
    }
}
__global__ void k_b_xpby(const double* z, double* p, const double* S, int64_t n) {
    const int k = blockIdx.y;
    if (S[G_STATE * kMrhs + k] != 0.0) return;
    const double b = S[G_BETA * kMrhs + k];
    const double* zk = z + k * n;
    double* pk = p + k * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pk[i] = zk[i] + b * pk[i];
}

// the block state of a handle, built on first use (two levels, additive, one system)
static BlockPcg& block_state(Handle& H, hipStream_t s) {
    if (H.bp) return *H.bp;
    Level& Lv = *H.lv[0];
    auto bp = std::make_unique<BlockPcg>();
    BlockPcg& B = *bp;
    const int64_t n = std::max<int64_t>(1, Lv.n), tot = std::max<int64_t>(1, Lv.hoffO[Lv.N]);
    const int64_t ptot = std::max<int64_t>(1, Lv.tpart.n);
    B.S.alloc(G_NSLOT * kMrhs);
    B.r.alloc(kMrhs * n);
    B.z.alloc(kMrhs * n);
    B.p.alloc(kMrhs * n);
    B.q.alloc(kMrhs * n);
    B.rloc.alloc(kMrhs * tot);
    B.yloc.alloc(kMrhs * tot);
    B.tpart.alloc(kMrhs * ptot);
    DD_HIP(hipHostMalloc(&B.hS, G_NSLOT * kMrhs * sizeof(double)));
    // the level's local-solve items, pointed at the column-blocked workspaces
    for (const TrmvItem& t : Lv.Tb.h)
        B.Tm.h.push_back(TrmvMItem<double>{t.W, t.ld, t.n, B.rloc.p + (t.x - Lv.rloc.p), B.yloc.p + (t.y - Lv.yloc.p),
                                           B.tpart.p + (t.part - Lv.tpart.p), tot, tot, ptot});
    for (const TrmvItem32& t : Lv.Tb32.h)
        B.Tm32.h.push_back(TrmvMItem<float>{t.W, t.ld, t.n, B.rloc.p + (t.x - Lv.rloc.p),
                                            B.yloc.p + (t.y - Lv.yloc.p), B.tpart.p + (t.part - Lv.tpart.p), tot, tot,
                                            ptot});
    if (!B.Tm.h.empty()) B.Tm.sync(s);
    if (!B.Tm32.h.empty()) B.Tm32.sync(s);
    H.bp = std::move(bp);
    return *H.bp;
}

// z_k = M r_k for K <= kMrhs columns (stride n): the steps of apply_level per
// column, with the local solves of all columns in one pass over the W_i.
// Columns with stopped[k] set (PCG columns that have stopped, whose z is not
// used again) skip the per-column coarse solve.
static void apply_block(Handle& H, const double* r, double* z, int K, hipStream_t s,
                        const std::vector<int>* stopped = nullptr) {
    Level& Lv = *H.lv[0];
    BlockPcg& B = block_state(H, s);
    const int64_t n = Lv.n, tot = Lv.hoffO[Lv.N];
    for (int k = 0; k < K; ++k) gather(r + k * n, Lv.omega_flat.p, tot, B.rloc.p + k * tot, s);
    if (!B.Tm32.h.empty()) trinv_apply_multi_vb(B.Tm32, K, s);
    if (!B.Tm.h.empty()) trinv_apply_multi_vb(B.Tm, K, s);
    for (int k = 0; k < K; ++k) {
        scatter_sum(B.rloc.p + k * tot, Lv.memb_ptr.p, Lv.memb.p, n, z + k * n, false, s);
        if (Lv.nC > 0 && !(stopped && (*stopped)[k])) {
            SubInfo S = Lv.sub();
            restrict_coarse(S, Lv.nC, r + k * n, Lv.yC.p, s);
            coarse_solve(H, 0, Lv.yC.p, s);
            prolong_coarse(S, Lv.offI.p, Lv.hoffI[Lv.N], Lv.yC.p, z + k * n, s);
        }
    }
}

static bool block_ok(const Handle& H) {
    return H.nsys() == 1 && H.lv.size() == 1 && H.opt.schwarz == DD_SCHWARZ_ADDITIVE;
}

// PCG on K <= kMrhs columns of b, x (stride n, x in/out) in lockstep
static int krylov_block(Handle& H, const double* b, double* x, int K, double rtol, int maxit, int* iters,
                        double* relres, hipStream_t s) {
    Level& Lv = *H.lv[0];
    const int64_t n = Lv.n;
    const CsrDev A = Lv.A();
    BlockPcg& B = block_state(H, s);
    double *r = B.r.p, *z = B.z.p, *p = B.p.p, *q = B.q.p, *S = B.S.p, *hS = B.hS;
    const dim3 vg(vgrid(n), K);
    // the start of krylov(), per column
    std::vector<double> bn(K), rn(K);
    dot(b, b, n, K, H.partial.p, S, s);
    d2h(hS, S, K, s);
    DD_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < K; ++k) {
        bn[k] = std::sqrt(hS[k]);
        DD_CHECK(std::isfinite(bn[k]), DD_ERR_NAN, "right-hand side contains NaN/Inf");
        if (bn[k] == 0.0) fill(x + k * n, n, 0.0, s);
    }
    spmv(A, x, r, K, s);
    for (int k = 0; k < K; ++k) hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b + k * n, r + k * n, n);
    dot(r, r, n, K, H.partial.p, S, s);
    d2h(hS, S, K, s);
    DD_HIP(hipStreamSynchronize(s));
    std::vector<int> state(K, 0);  // 0 running, 1 converged, 2 maxit, 3 NaN
    for (int k = 0; k < K; ++k) {
        rn[k] = std::sqrt(hS[k]);
        if (bn[k] == 0.0 || rn[k] <= rtol * bn[k]) state[k] = 1;
        else if (maxit <= 0) state[k] = 2;
    }
    std::vector<int> its(K, 0);
    if (std::count(state.begin(), state.end(), 0) > 0) {
        apply_block(H, r, z, K, s);
        DD_HIP(hipMemcpyAsync(p, z, K * n * sizeof(double), hipMemcpyDeviceToDevice, s));
        dot(r, z, n, K, H.partial.p, S + G_RZ * kMrhs, s);
        d2h(hS, S, G_NSLOT * kMrhs, s);
        DD_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < K; ++k) {
            for (int g = 0; g < G_NSLOT; ++g)
                if (g != G_RZ) hS[g * kMrhs + k] = 0.0;
            hS[G_THR * kMrhs + k] = rtol * bn[k];
            hS[G_MAXIT * kMrhs + k] = maxit;
            hS[G_STATE * kMrhs + k] = state[k];
        }
        h2d(S, hS, G_NSLOT * kMrhs, s);
        std::vector<int> stopped(K);
        for (int k = 0; k < K; ++k) stopped[k] = state[k] != 0;
        int batch = 2;
        for (;;) {
            for (int j = 0; j < batch; ++j) {
                spmv(A, p, q, K, s);
                dot(p, q, n, K, H.partial.p, S + G_PQ * kMrhs, s);
                hipLaunchKernelGGL(k_b_alpha, dim3(1), dim3(kMrhs), 0, s, S, K);
                hipLaunchKernelGGL(k_b_axpy2, vg, dim3(256), 0, s, x, r, p, q, S, n);
                dot(r, r, n, K, H.partial.p, S + G_RN2 * kMrhs, s);
                hipLaunchKernelGGL(k_b_check, dim3(1), dim3(kMrhs), 0, s, S, K);
                apply_block(H, r, z, K, s, &stopped);
                dot(r, z, n, K, H.partial.p, S + G_RZN * kMrhs, s);
                hipLaunchKernelGGL(k_b_beta, dim3(1), dim3(kMrhs), 0, s, S, K);
                hipLaunchKernelGGL(k_b_xpby, vg, dim3(256), 0, s, z, p, S, n);
                launch_check("block_pcg");
            }
            d2h(hS, S, G_NSLOT * kMrhs, s);
            DD_HIP(hipStreamSynchronize(s));
            bool running = false;
            for (int k = 0; k < K; ++k) {
                stopped[k] = hS[G_STATE * kMrhs + k] != 0.0;
                running = running || !stopped[k];
            }
            if (!running) break;
            batch = std::min(8, batch * 2);
        }
        for (int k = 0; k < K; ++k) {
            DD_CHECK(hS[G_STATE * kMrhs + k] != 3.0, DD_ERR_NAN, "PCG produced NaN");
            if (state[k] == 0) {
                its[k] = (int)hS[G_ITS * kMrhs + k];
                state[k] = (int)hS[G_STATE * kMrhs + k];
            }
        }
    }
    // true residuals at exit
    spmv(A, x, r, K, s);
    for (int k = 0; k < K; ++k) hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b + k * n, r + k * n, n);
    dot(r, r, n, K, H.partial.p, S, s);
    d2h(hS, S, K, s);
    DD_HIP(hipStreamSynchronize(s));
    int rc = DD_OK;
    for (int k = 0; k < K; ++k) {
        const double rel = bn[k] == 0.0 ? 0.0 : std::sqrt(hS[k]) / bn[k];
        DD_CHECK(std::isfinite(rel), DD_ERR_NAN, "PCG produced NaN");
        iters[k] = its[k];
        relres[k] = rel;
        if (state[k] != 1) rc = DD_WARN_MAXIT;
    }
    return rc;
}

// ---------------------------------------------------------------------------
// Right-preconditioned GMRES(restart) (R12): Arnoldi on A M with classical
// Gram-Schmidt applied twice, so each orthogonalisation is two tall-skinny
// products with the basis (V^T w, then w -= V h) instead of j dependent dot
// products; the Hessenberg column comes to the host once per step, where the
// Givens rotations and the small triangular solve run.
// ---------------------------------------------------------------------------
// part[c * gridDim.x + blockIdx.x] = sum over the block's rows of V[i + c ld] w[i],
// c < k; four columns per pass share each w[i] load
__global__ __launch_bounds__(256) void k_gemv_t_part(const double* V, int64_t ld, int k, const double* w, int64_t n,
                                                     double* part) {
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int c0 = 0; c0 < k; c0 += 4) {
        const int nc = k - c0 < 4 ? k - c0 : 4;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
            const double wi = w[i];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < nc) a[c] += V[i + (int64_t)(c0 + c) * ld] * wi;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double v = a[c];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) red[c][wv] = v;
        }
        __syncthreads();
        if (threadIdx.x < nc)
            part[(int64_t)(c0 + threadIdx.x) * gridDim.x + blockIdx.x] =
                red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        __syncthreads();
    }
}
// out[c] = sum_b part[c * nb + b], fixed order; a wave per column
__global__ __launch_bounds__(256) void k_gemv_t_final(const double* part, int nb, int k, double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = wv; c < k; c += 4) {
        double v = 0.0;
        for (int b = lane; b < nb; b += 64) v += part[(int64_t)c * nb + b];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) out[c] = v;
    }
}
// w := (accumulate ? w : 0) + alpha V h, V n x k (ld), h on the device (k <= kMaxRestart + 1)
__global__ __launch_bounds__(256) void k_gemv_n(const double* V, int64_t ld, int k, const double* h, double alpha,
                                                double* w, int64_t n, int accumulate) {
    __shared__ double hs[kMaxRestart + 1];
    for (int c = threadIdx.x; c < k; c += blockDim.x) hs[c] = h[c];
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < k; ++c) acc += V[i + (int64_t)c * ld] * hs[c];
        w[i] = (accumulate ? w[i] : 0.0) + alpha * acc;
    }
}
__global__ void k_scale_to(const double* x, double a, double* y, int64_t n) {  // y = a x
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}

static void gemv_t(const double* V, int64_t n, int k, const double* w, double* part, double* out, hipStream_t s) {
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kGemvBlocks, (n + 255) / 256));
    hipLaunchKernelGGL(k_gemv_t_part, dim3(nb), dim3(256), 0, s, V, n, k, w, n, part);
    hipLaunchKernelGGL(k_gemv_t_final, dim3(1), dim3(256), 0, s, part, nb, k, out);
}

// GMRES(restart) on the matrix of level m, right-preconditioned by level m's
// M (additive or deflated), x holds x0 on entry.  A cycle ends when the
// Arnoldi estimate |g_{j+1}| reaches rtol ||b||, after `restart` steps, on
// breakdown or at maxit steps in total; the true residual then starts the next
// cycle and is the one reported.  The preconditioned directions z_j = M v_j
// are kept and x += [z_1 ... z_k] y (the flexible form): for a fixed M this is
// the same iterate as x += M (V y) and saves that apply at the end of every
// cycle; it also serves a preconditioner that varies (inner iterative coarse
// solves) or is linear only up to FP32 rounding (FP32 local solves).
static int gmres(Handle& H, size_t m, const double* b, double* x, double rtol, int maxit, int restart, int* iters,
                 double* relres, hipStream_t s) {
    Level& Lv = *H.lv[m];
    const int64_t n = Lv.n;
    const CsrDev A = Lv.A();
    GmresWork& G = Lv.gm;
    G.ensure(n, restart);
    double *V = G.V.p, *w = G.w.p, *hd = G.h.p, *hp = G.hp;
    double* yd = hd + kHcol;  // device copy of the cycle's y
    double* yh = hp + kHcol;  // pinned host copy
    const int g1 = vgrid(n);
    const double bn = std::sqrt(dot_host(H, b, b, n, s));
    DD_CHECK(std::isfinite(bn), DD_ERR_NAN, "right-hand side contains NaN/Inf");
    if (bn == 0.0) {
        fill(x, n, 0.0, s);
        *iters = 0;
        *relres = 0.0;
        return DD_OK;
    }
    spmv(A, x, w, 1, s);
    hipLaunchKernelGGL(k_sub, dim3(g1), dim3(256), 0, s, b, w, n);  // w = b - A x
    double beta = std::sqrt(dot_host(H, w, w, n, s));
    DD_CHECK(std::isfinite(beta), DD_ERR_NAN, "GMRES produced NaN");
    const int ldh = restart + 1;
    std::vector<double> Hm((size_t)ldh * restart), cs(restart), sn(restart), g(restart + 1);
    int its = 0;
    while (beta > rtol * bn && its < maxit) {
        hipLaunchKernelGGL(k_scale_to, dim3(g1), dim3(256), 0, s, w, 1.0 / beta, V, n);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < restart; ++j) {
            const double* vj = V + (int64_t)j * n;
            double* zj = G.Zf.p + (int64_t)j * n;
            apply_level(H, m, vj, zj, s);
            spmv(A, zj, w, 1, s);
            // two passes of classical Gram-Schmidt against v_0 .. v_j
            gemv_t(V, n, j + 1, w, G.part.p, hd, s);
            hipLaunchKernelGGL(k_gemv_n, dim3(g1), dim3(256), 0, s, V, n, j + 1, hd, -1.0, w, n, 1);
            gemv_t(V, n, j + 1, w, G.part.p, hd + kMaxRestart + 1, s);
            hipLaunchKernelGGL(k_gemv_n, dim3(g1), dim3(256), 0, s, V, n, j + 1, hd + kMaxRestart + 1, -1.0, w, n, 1);
            dot(w, w, n, 1, H.partial.p, hd + 2 * (kMaxRestart + 1), s);
            DD_HIP(hipMemcpyAsync(hp, hd, kHcol * sizeof(double), hipMemcpyDeviceToHost, s));
            DD_HIP(hipStreamSynchronize(s));
            double* col = Hm.data() + (size_t)j * ldh;
            for (int i = 0; i <= j; ++i) col[i] = hp[i] + hp[kMaxRestart + 1 + i];
            const double hn = std::sqrt(hp[2 * (kMaxRestart + 1)]);
            DD_CHECK(std::isfinite(hn), DD_ERR_NAN, "GMRES produced NaN");
            col[j + 1] = hn;
            if (hn > 0.0)
                hipLaunchKernelGGL(k_scale_to, dim3(g1), dim3(256), 0, s, w, 1.0 / hn, V + (int64_t)(j + 1) * n, n);
            for (int i = 0; i < j; ++i) {  // earlier rotations on the new column
                const double a = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = a;
            }
            const double d = std::hypot(col[j], col[j + 1]);
            DD_CHECK(d > 0.0, DD_ERR_NAN, "GMRES breakdown (singular Hessenberg matrix)");
            cs[j] = col[j] / d;
            sn[j] = col[j + 1] / d;
            col[j] = d;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++its;
            k = j + 1;
            if (std::fabs(g[j + 1]) <= rtol * bn || its >= maxit || sn[j] == 0.0) break;
        }
        // y = R^{-1} g by back substitution, then the update of x
        for (int i = k - 1; i >= 0; --i) {
            double v = g[i];
            for (int l = i + 1; l < k; ++l) v -= Hm[(size_t)l * ldh + i] * yh[l];
            yh[i] = v / Hm[(size_t)i * ldh + i];
        }
        DD_HIP(hipMemcpyAsync(yd, yh, k * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_gemv_n, dim3(g1), dim3(256), 0, s, G.Zf.p, n, k, yd, 1.0, x, n, 1);
        spmv(A, x, w, 1, s);
        hipLaunchKernelGGL(k_sub, dim3(g1), dim3(256), 0, s, b, w, n);
        beta = std::sqrt(dot_host(H, w, w, n, s));  // synchronises: yh may be rewritten next cycle
        DD_CHECK(std::isfinite(beta), DD_ERR_NAN, "GMRES produced NaN");
    }
    *iters = its;
    *relres = beta / bn;
    return beta <= rtol * bn ? DD_OK : DD_WARN_MAXIT;
}

// ---------------------------------------------------------------------------
// One PCG per system of a batch (dd_setup_batch), run in lockstep on the
// union vector: every dot product is per system (segmented reduction), alpha
// and beta are per system, and a system that has converged takes alpha = 0 so
// its iterate stays put while the others go on.  The preconditioner of the
// union is block diagonal over the systems, so each system sees its own PCG.
// ---------------------------------------------------------------------------
__global__ void k_axpy2_seg(double* x, double* r, const double* p, const double* q, const double* alpha,
                            const int32_t* sid, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = alpha[sid[i]];
        x[i] += a * p[i];
        r[i] -= a * q[i];
    }
}
__global__ void k_xpby_seg(const double* z, double* p, const double* beta, const int32_t* sid, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta[sid[i]] * p[i];
}

// the systems' dof ranges on level m of a batch (level 0: the handle's)
struct SegView {
    const std::vector<int64_t>* off;
    const int64_t* doff;
    const int32_t* sid;
};
static SegView seg_of(Handle& H, size_t m) {
    const size_t want = (size_t)H.nsys() + 1;
    if (m == 0) {
        DD_CHECK(H.sys_off.size() == want && H.dsys_off.p && H.sys_id.p, DD_ERR_INTERNAL,
                 "batch handle without system ranges on level 0");
        return SegView{&H.sys_off, H.dsys_off.p, H.sys_id.p};
    }
    Level& Lv = *H.lv[m];
    DD_CHECK(Lv.hseg.size() == want && Lv.dseg.p && Lv.seg_id.p, DD_ERR_INTERNAL,
             "batch level without per-system ranges");
    return SegView{&Lv.hseg, Lv.dseg.p, Lv.seg_id.p};
}

static std::vector<double> dot_sys(Handle& H, const SegView& g, const double* x, const double* y, hipStream_t s) {
    const int ns = H.nsys();
    dot_seg(x, y, g.doff, ns, H.partial.p, H.dots.p, s);
    DD_HIP(hipMemcpyAsync(H.hpin, H.dots.p, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    DD_HIP(hipStreamSynchronize(s));
    return std::vector<double>(H.hpin, H.hpin + ns);
}
// per-system scalars to the device (slot 0: alpha, slot 1: beta); the pinned
// slot is not rewritten before a later stream synchronisation
static const double* put_sys(Handle& H, const std::vector<double>& v, int slot, hipStream_t s) {
    const int ns = H.nsys();
    double* h = H.hscal + (size_t)slot * ns;
    std::copy(v.begin(), v.end(), h);
    double* d = H.dscal.p + (size_t)slot * ns;
    DD_HIP(hipMemcpyAsync(d, h, ns * sizeof(double), hipMemcpyHostToDevice, s));
    return d;
}

// One PCG per system on level m of a batch (the outer solve on level 0, the
// inner coarse solves below it); iters and relres (nsys entries) may be null.
// true_res: the true residual of every system is computed at exit.
static int krylov_seg(Handle& H, size_t m, const double* b, double* x, double rtol, int maxit, bool flexible,
                      bool true_res, int* iters, double* relres, hipStream_t s) {
    Level& Lv = *H.lv[m];
    const int64_t n = Lv.n;
    const int ns = H.nsys();
    const CsrDev A = Lv.A();
    const SegView g = seg_of(H, m);
    const std::vector<int64_t>& off = *g.off;
    double *r = Lv.kr.p, *z = Lv.kz.p, *p = Lv.kp.p, *q = Lv.kq.p, *ro = Lv.kro.p;
    std::vector<double> bn = dot_sys(H, g, b, b, s);
    for (int k = 0; k < ns; ++k) {
        DD_CHECK(std::isfinite(bn[k]), DD_ERR_NAN, "right-hand side contains NaN/Inf");
        bn[k] = std::sqrt(bn[k]);
        if (bn[k] == 0.0 && off[k + 1] > off[k]) fill(x + off[k], off[k + 1] - off[k], 0.0, s);
    }
    spmv(A, x, r, 1, s);
    hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b, r, n);
    std::vector<double> rn = dot_sys(H, g, r, r, s);
    std::vector<int> its(ns, 0);
    std::vector<char> conv(ns, 0);
    int left = 0;
    for (int k = 0; k < ns; ++k) {
        rn[k] = std::sqrt(rn[k]);
        conv[k] = (bn[k] == 0.0 || rn[k] <= rtol * bn[k]) ? 1 : 0;
        left += conv[k] ? 0 : 1;
    }
    if (left) {
        apply_level(H, m, r, z, s);
        DD_HIP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        std::vector<double> rz = dot_sys(H, g, r, z, s);
        std::vector<double> alpha(ns), beta(ns);
        for (int it = 1; it <= maxit && left; ++it) {
            spmv(A, p, q, 1, s);
            const std::vector<double> pq = dot_sys(H, g, p, q, s);
            for (int k = 0; k < ns; ++k) {
                alpha[k] = conv[k] ? 0.0 : rz[k] / pq[k];
                DD_CHECK(std::isfinite(alpha[k]), DD_ERR_NAN, "PCG produced NaN");
            }
            if (flexible) DD_HIP(hipMemcpyAsync(ro, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_axpy2_seg, dim3(vgrid(n)), dim3(256), 0, s, x, r, p, q, put_sys(H, alpha, 0, s),
                               g.sid, n);
            rn = dot_sys(H, g, r, r, s);
            for (int k = 0; k < ns; ++k) {
                if (conv[k]) continue;
                its[k] = it;
                if (std::sqrt(rn[k]) <= rtol * bn[k]) {
                    conv[k] = 1;
                    --left;
                }
            }
            if (!left) break;
            apply_level(H, m, r, z, s);
            if (flexible) {
                hipLaunchKernelGGL(k_diff, dim3(vgrid(n)), dim3(256), 0, s, r, ro, q, n);  // q := r - r_old
                const std::vector<double> zq = dot_sys(H, g, z, q, s);
                for (int k = 0; k < ns; ++k) beta[k] = conv[k] ? 0.0 : zq[k] / rz[k];
                rz = dot_sys(H, g, r, z, s);
            } else {
                const std::vector<double> rzn = dot_sys(H, g, r, z, s);
                for (int k = 0; k < ns; ++k) beta[k] = conv[k] ? 0.0 : rzn[k] / rz[k];
                rz = rzn;
            }
            hipLaunchKernelGGL(k_xpby_seg, dim3(vgrid(n)), dim3(256), 0, s, z, p, put_sys(H, beta, 1, s), g.sid,
                               n);
        }
    }
    if (true_res) {  // else the recurrence residual r
        spmv(A, x, r, 1, s);
        hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b, r, n);
    }
    const std::vector<double> tr = dot_sys(H, g, r, r, s);
    bool all = true;
    for (int k = 0; k < ns; ++k) {
        const double rel = bn[k] > 0.0 ? std::sqrt(tr[k]) / bn[k] : 0.0;
        DD_CHECK(std::isfinite(rel), DD_ERR_NAN, "PCG produced NaN");
        if (iters) iters[k] = its[k];
        if (relres) relres[k] = rel;
        all = all && conv[k];
    }
    return all ? DD_OK : DD_WARN_MAXIT;
}

// The graph PCG of a batch handle (two levels, additive): one PCG per system as
// in krylov_seg, every system's scalars on the device (S[slot * ns + k]) and
// the same per-system kernels, so that each system's iterates are those of the
// host loop bit for bit; a system that has stopped takes zero steps
// (alpha = beta = 0), as it does there.
__global__ void k_s_alpha(double* S, int ns) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns) return;
    double* a = S + G_ALPHA * ns;
    if (S[G_STATE * ns + k] != 0.0) {
        a[k] = 0.0;
        return;
    }
    const double v = S[G_RZ * ns + k] / S[G_PQ * ns + k];
    if (!isfinite(v)) {
        S[G_STATE * ns + k] = 3.0;
        a[k] = 0.0;
        return;
    }
    a[k] = v;
}
__global__ void k_s_check(double* S, int ns) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns || S[G_STATE * ns + k] != 0.0) return;
    S[G_ITS * ns + k] += 1.0;
    if (sqrt(S[G_RN2 * ns + k]) <= S[G_THR * ns + k]) S[G_STATE * ns + k] = 1.0;
    else if (S[G_ITS * ns + k] >= S[G_MAXIT * ns + k]) S[G_STATE * ns + k] = 2.0;
}
__global__ void k_s_beta(double* S, int ns) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns) return;
    if (S[G_STATE * ns + k] != 0.0) {
        S[G_BETA * ns + k] = 0.0;
        return;
    }
    S[G_BETA * ns + k] = S[G_RZN * ns + k] / S[G_RZ * ns + k];
    S[G_RZ * ns + k] = S[G_RZN * ns + k];
}

static void graph_iteration_seg(Handle& H, double* S, int ns, hipStream_t s) {
    Level& Lv = *H.lv[0];
    const int64_t n = Lv.n;
    const CsrDev A = Lv.A();
    const SegView g = seg_of(H, 0);
    double *x = Lv.kx.p, *r = Lv.kr.p, *z = Lv.kz.p, *p = Lv.kp.p, *q = Lv.kq.p;
    const int gs = ceil_div(ns, 64);
    spmv(A, p, q, 1, s);
    dot_seg(p, q, g.doff, ns, H.partial.p, S + G_PQ * ns, s);
    hipLaunchKernelGGL(k_s_alpha, dim3(gs), dim3(64), 0, s, S, ns);
    hipLaunchKernelGGL(k_axpy2_seg, dim3(vgrid(n)), dim3(256), 0, s, x, r, p, q, S + G_ALPHA * ns, g.sid, n);
    dot_seg(r, r, g.doff, ns, H.partial.p, S + G_RN2 * ns, s);
    hipLaunchKernelGGL(k_s_check, dim3(gs), dim3(64), 0, s, S, ns);
    apply_level(H, 0, r, z, s);
    dot_seg(r, z, g.doff, ns, H.partial.p, S + G_RZN * ns, s);
    hipLaunchKernelGGL(k_s_beta, dim3(gs), dim3(64), 0, s, S, ns);
    hipLaunchKernelGGL(k_xpby_seg, dim3(vgrid(n)), dim3(256), 0, s, z, p, S + G_BETA * ns, g.sid, n);
    launch_check("graph_pcg_batch");
}

static int krylov_graph_seg(Handle& H, const double* b, double* xio, double rtol, int maxit, int* iters,
                            double* relres, hipStream_t s) {
    Level& Lv = *H.lv[0];
    const int64_t n = Lv.n;
    const int ns = H.nsys();
    const CsrDev A = Lv.A();
    const SegView g = seg_of(H, 0);
    const std::vector<int64_t>& off = *g.off;
    if (!H.gp || H.gp->chunk != H.opt.graph_pcg || H.gp->ns != ns) {
        H.gp = std::make_unique<GraphPcg>();
        GraphPcg& G = *H.gp;
        G.chunk = H.opt.graph_pcg;
        G.ns = ns;
        G.S.alloc((size_t)G_NSLOT * ns);
        DD_HIP(hipHostMalloc(&G.hS, (size_t)G_NSLOT * ns * sizeof(double)));
        DD_HIP(hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking));
        DD_HIP(hipStreamBeginCapture(G.cs, hipStreamCaptureModeThreadLocal));
        try {
            graph_iteration_seg(H, G.S.p, ns, G.cs);
        } catch (...) {
            hipGraph_t gr = nullptr;
            (void)hipStreamEndCapture(G.cs, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            H.gp.reset();
            throw;
        }
        DD_HIP(hipStreamEndCapture(G.cs, &G.graph));
        DD_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
    }
    GraphPcg& G = *H.gp;
    double *x = Lv.kx.p, *r = Lv.kr.p, *z = Lv.kz.p, *p = Lv.kp.p;
    DD_HIP(hipMemcpyAsync(x, xio, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    // the start as in krylov_seg
    std::vector<double> bn = dot_sys(H, g, b, b, s);
    for (int k = 0; k < ns; ++k) {
        DD_CHECK(std::isfinite(bn[k]), DD_ERR_NAN, "right-hand side contains NaN/Inf");
        bn[k] = std::sqrt(bn[k]);
        if (bn[k] == 0.0 && off[k + 1] > off[k]) fill(x + off[k], off[k + 1] - off[k], 0.0, s);
    }
    spmv(A, x, r, 1, s);
    hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b, r, n);
    std::vector<double> rn = dot_sys(H, g, r, r, s);
    std::vector<int> its(ns, 0);
    std::vector<char> conv(ns, 0);
    int left = 0;
    for (int k = 0; k < ns; ++k) {
        rn[k] = std::sqrt(rn[k]);
        conv[k] = (bn[k] == 0.0 || rn[k] <= rtol * bn[k]) ? 1 : 0;
        left += conv[k] ? 0 : 1;
    }
    if (left && maxit > 0) {
        apply_level(H, 0, r, z, s);
        DD_HIP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        const std::vector<double> rz = dot_sys(H, g, r, z, s);
        double* hS = G.hS;
        std::fill(hS, hS + (size_t)G_NSLOT * ns, 0.0);
        for (int k = 0; k < ns; ++k) {
            hS[G_RZ * ns + k] = rz[k];
            hS[G_THR * ns + k] = rtol * bn[k];
            hS[G_MAXIT * ns + k] = maxit;
            hS[G_STATE * ns + k] = conv[k] ? 1.0 : 0.0;
        }
        h2d(G.S.p, hS, (size_t)G_NSLOT * ns, s);
        // batches of replays between host checks, sized from the slowest system's
        // residual contraction
        int batch = std::min(2, G.chunk);
        std::vector<double> rprev(rn);
        for (;;) {
            for (int j = 0; j < batch; ++j) DD_HIP(hipGraphLaunch(G.exec, s));
            d2h(hS, G.S.p, (size_t)G_NSLOT * ns, s);
            DD_HIP(hipStreamSynchronize(s));
            bool all = true;
            double est = 1.0;
            for (int k = 0; k < ns; ++k) {
                if (hS[G_STATE * ns + k] != 0.0) continue;
                all = false;
                const double rcur = std::sqrt(hS[G_RN2 * ns + k]);
                const double rate = std::pow(rcur / rprev[k], 1.0 / batch);
                rprev[k] = rcur;
                double e = G.chunk;
                if (rate > 0.0 && rate < 1.0) e = std::log(hS[G_THR * ns + k] / rcur) / std::log(rate);
                est = std::max(est, e);
            }
            if (all) break;
            batch = (int)std::max(1.0, std::min<double>(G.chunk, std::floor(est)));
        }
        for (int k = 0; k < ns; ++k) {
            DD_CHECK(hS[G_STATE * ns + k] != 3.0, DD_ERR_NAN, "PCG produced NaN");
            its[k] = (int)hS[G_ITS * ns + k];
            conv[k] = conv[k] || hS[G_STATE * ns + k] == 1.0;
        }
    }
    // true residual at exit
    spmv(A, x, r, 1, s);
    hipLaunchKernelGGL(k_sub, dim3(vgrid(n)), dim3(256), 0, s, b, r, n);
    const std::vector<double> tr = dot_sys(H, g, r, r, s);
    bool all = true;
    for (int k = 0; k < ns; ++k) {
        const double rel = bn[k] > 0.0 ? std::sqrt(tr[k]) / bn[k] : 0.0;
        DD_CHECK(std::isfinite(rel), DD_ERR_NAN, "PCG produced NaN");
        if (iters) iters[k] = its[k];
        if (relres) relres[k] = rel;
        all = all && conv[k];
    }
    DD_HIP(hipMemcpyAsync(xio, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    return all ? DD_OK : DD_WARN_MAXIT;
}

__global__ void k_copy_add_i32(const int32_t* src, int32_t* dst, int64_t n, int64_t add) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (int32_t)(src[i] + add);
}
__global__ void k_set_i32(int32_t* dst, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = v;
}

// k_c of the bound of Sec. 3.2: greedy colouring, subdomains in index order,
// each taking the smallest colour none of its neighbours has, on the graph
// i ~ j iff A(Omega_i, Omega_j) != 0.  The columns of the rows Omega_i are
// exactly Omega~_i = [Omega_i, Delta_i] (every dof of Omega_i has its
// diagonal entry, every dof of Delta_i a neighbour in Omega_i), so i ~ j iff
// Omega~_i meets Omega_j.
static int coloring_kc(const Level& L) {
    const int N = L.N;
    const auto ext = to_host(L.ext.p, (size_t)L.hoffE[N], nullptr);
    std::vector<int64_t> cnt(L.n + 1, 0);  // subdomains whose Omega holds each dof (CSR)
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < L.ni[j]; ++k) cnt[ext[L.hoffE[j] + k] + 1] += 1;
    for (int64_t g = 0; g < L.n; ++g) cnt[g + 1] += cnt[g];
    std::vector<int32_t> who(cnt[L.n]);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < L.ni[j]; ++k) who[pos[ext[L.hoffE[j] + k]]++] = j;
    std::vector<int> color(N, -1), mark(N + 1, -1);
    int kc = 0;
    for (int i = 0; i < N; ++i) {
        for (int k = 0; k < L.nt[i]; ++k) {
            const int64_t g = ext[L.hoffE[i] + k];
            for (int64_t q = cnt[g]; q < cnt[g + 1]; ++q) {
                const int j = who[q];
                if (j != i && color[j] >= 0) mark[color[j]] = i;
            }
        }
        int c = 0;
        while (mark[c] == i) ++c;
        color[i] = c;
        kc = std::max(kc, c + 1);
    }
    return kc;
}

}  // namespace dd

// ===========================================================================
// C-ABI
// ===========================================================================
using namespace dd;

struct dd_handle_s {
    Handle h;
};

#define DD_GUARD_BEGIN try {
#define DD_GUARD_END                                                  \
    }                                                                 \
    catch (const dd::Error& e) {                                      \
        if (std::getenv("DD_VERBOSE")) fprintf(stderr, "dd: %s\n", e.what()); \
        return e.code;                                                \
    }                                                                 \
    catch (const std::bad_alloc&) {                                   \
        return DD_ERR_OOM;                                            \
    }                                                                 \
    catch (...) {                                                     \
        return DD_ERR_INTERNAL;                                       \
    }

namespace dd {
Meter& meter() {
    static Meter m;
    return m;
}
// ---------------------------------------------------------------------------
// Device cache behind DBuf.  Requests are rounded to a size class (4 KiB steps
// below 64 KiB, 2 MiB steps below 1 GiB, then 1/16 of the power of two below
// the size) and served by the smallest cached block of the same device whose
// class is at most 25 % larger.  A freed block may still be in use by work
// queued before its release, so it is handed out again only after a device
// synchronisation that follows the release (one is made here when needed).
// The cache holds at most DD_DEVICE_CACHE_GB GiB (default 96, 0 disables it);
// beyond that, or on dd_trim_device_cache, blocks go back to hipFree, and a
// failed hipMalloc empties the cache of that device and is retried once.
// ---------------------------------------------------------------------------
namespace {
struct CacheBlock {
    size_t cls;
    int dev;
    uint64_t epoch;
};
struct DeviceCache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<std::pair<void*, uint64_t>>> free_;  // (dev, cls) -> blocks
    std::unordered_map<void*, CacheBlock> live_;
    uint64_t epoch = 1;  // advanced by every device synchronisation made here
    size_t cached = 0, cap = 0;
    DeviceCache() {
        const char* e = std::getenv("DD_DEVICE_CACHE_GB");
        const double gb = e ? std::atof(e) : 96.0;
        cap = gb > 0.0 ? (size_t)(gb * (double)(1ull << 30)) : 0;
    }
};
DeviceCache& device_cache() {
    static DeviceCache* c = new DeviceCache;  // never destroyed: the process teardown releases device memory
    return *c;
}
size_t size_class(size_t b) {
    if (b < (64u << 10)) return (b + 4095) / 4096 * 4096;
    if (b < (1ull << 30)) return (b + (2u << 20) - 1) / (2u << 20) * (2u << 20);
    const size_t step = (size_t(1) << (63 - __builtin_clzll(b))) / 16;
    return (b + step - 1) / step * step;
}
// every cached block of device `dev` back to hipFree (caller holds the lock)
void trim_locked(DeviceCache& c, int dev) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    for (auto it = c.free_.begin(); it != c.free_.end();) {
        if (it->first.first != dev) { ++it; continue; }
        for (auto& b : it->second) {
            (void)hipFree(b.first);
            c.cached -= it->first.second;
        }
        it = c.free_.erase(it);
    }
    if (cur != dev) (void)hipSetDevice(cur);
}
}  // namespace

void* dd::dev_alloc(size_t bytes) {
    DeviceCache& c = device_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    int dev = 0;
    DD_HIP(hipGetDevice(&dev));
    const size_t cls = size_class(bytes);
    auto it = c.free_.lower_bound({dev, cls});
    if (it != c.free_.end() && it->first.first == dev && it->first.second <= cls + cls / 4) {
        auto& v = it->second;
        const auto blk = v.back();
        if (blk.second >= c.epoch) {  // released since the last synchronisation
            DD_HIP(hipDeviceSynchronize());
            ++c.epoch;
        }
        v.pop_back();
        const size_t got = it->first.second;
        if (v.empty()) c.free_.erase(it);
        c.cached -= got;
        c.live_[blk.first] = CacheBlock{got, dev, 0};
        return blk.first;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cls);
    if (e == hipErrorOutOfMemory && c.cached > 0) {
        (void)hipGetLastError();
        trim_locked(c, dev);
        e = hipMalloc(&p, cls);
    }
    DD_HIP(e);
    c.live_[p] = CacheBlock{cls, dev, 0};
    return p;
}

void dd::dev_free(void* p, size_t) noexcept {
    DeviceCache& c = device_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live_.find(p);
    if (it == c.live_.end()) return;
    const CacheBlock b = it->second;
    c.live_.erase(it);
    if (c.cached + b.cls > c.cap) {
        (void)hipFree(p);
        return;
    }
    try {
        c.free_[{b.dev, b.cls}].push_back({p, c.epoch});
        c.cached += b.cls;
    } catch (...) {
        (void)hipFree(p);
    }
}

// ---------------------------------------------------------------------------
// launch-mapping autotuner of launch_tiles
// ---------------------------------------------------------------------------
namespace {
struct TuneCand {
    int mode, grid;
    double ms = 0.0;
    double tiles = 0.0;
    int n = 0;
};
struct TuneEntry {
    std::vector<TuneCand> cand;
    int next = 0;
    int best = -1;
    struct Pending {
        int cand;
        hipEvent_t e0, e1;
        int64_t tiles;
    };
    std::vector<Pending> pending;
};
struct Tuner {
    std::mutex mu;
    std::unordered_map<std::string, TuneEntry> table;
    std::vector<hipEvent_t> events;  // recycled
    int enabled = -1;
};
Tuner& tuner() {
    static Tuner t;
    return t;
}
constexpr int kTuneSamples = 3;
constexpr double kTuneMs = 0.5;
constexpr double kTuneCheapMs = 0.1;
constexpr int kTileCounters = 4096;
}  // namespace

static __device__ int tile_counters[kTileCounters];

__global__ void k_zero_counter(int* c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

int* tile_counter(int n) {
    static std::mutex mu;
    static int* base[64] = {};
    static unsigned next = 0;
    int dev = 0;
    DD_HIP(hipGetDevice(&dev));
    DD_CHECK(dev >= 0 && dev < 64, DD_ERR_INTERNAL, "device index beyond the counter table");
    std::lock_guard<std::mutex> lk(mu);
    if (!base[dev]) {
        void* p = nullptr;
        DD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(tile_counters)));
        base[dev] = static_cast<int*>(p);
    }
    // n consecutive slots, never wrapping past the end of the array
    const unsigned slot = (next % (kTileCounters / kXcds)) * kXcds;
    next++;
    DD_CHECK(n >= 1 && n <= kXcds, DD_ERR_INTERNAL, "tile counter request beyond one slot");
    return base[dev] + slot;
}

hipEvent_t tile_event() {
    Tuner& T = tuner();
    std::lock_guard<std::mutex> lk(T.mu);
    if (!T.events.empty()) {
        hipEvent_t e = T.events.back();
        T.events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    DD_HIP(hipEventCreate(&e));
    return e;
}

// completed samples of an entry into its candidates; decide once every
// candidate is measured well enough: kTuneSamples samples, or one sample for a
// candidate whose samples total kTuneMs (a long launch times reliably once),
// or one sample each when the fastest candidate averages under kTuneCheapMs
// (the choice is then worth little, and gross differences show in one
// sample).  Called with the lock held.
static void tune_poll(Tuner& T, TuneEntry& E) {
    std::vector<TuneEntry::Pending> keep;
    for (auto& q : E.pending) {
        if (hipEventQuery(q.e1) != hipSuccess) {
            keep.push_back(q);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, q.e0, q.e1) == hipSuccess) {
            TuneCand& c = E.cand[q.cand];
            c.ms += ms;
            c.tiles += (double)q.tiles;
            c.n += 1;
        }
        T.events.push_back(q.e0);
        T.events.push_back(q.e1);
    }
    E.pending.swap(keep);
    if (E.best >= 0) return;
    int best = -1;
    double bt = 0.0;
    double fastest = 1e300;
    for (const TuneCand& c : E.cand) {
        if (c.n < 1) return;
        fastest = std::min(fastest, c.ms / c.n);
    }
    const bool cheap = fastest < kTuneCheapMs;
    for (size_t c = 0; c < E.cand.size(); ++c) {
        if (!cheap && E.cand[c].n < kTuneSamples && E.cand[c].ms < kTuneMs) return;
        const double per = E.cand[c].ms / std::max(1.0, E.cand[c].tiles);
        if (best < 0 || per < bt) {
            best = (int)c;
            bt = per;
        }
    }
    E.best = best;
}

TileChoice tile_choice(const char* name, bool xcd_ok, int max_grid, hipStream_t s) {
    Tuner& T = tuner();
    const TileChoice fixed{xcd_ok ? TM_XCD : TM_STATIC, max_grid, -1};
    std::lock_guard<std::mutex> lk(T.mu);
    if (T.enabled < 0) {
        const char* e = std::getenv("DD_AUTOTUNE");
        T.enabled = (e && std::atoi(e) == 0) ? 0 : 1;
    }
    if (!T.enabled) return fixed;
    TuneEntry& E = T.table[name];
    if (E.cand.empty()) {
        E.cand.push_back(TuneCand{fixed.mode, max_grid});
        E.cand.push_back(TuneCand{TM_STATIC, std::max(256, max_grid / 2)});
        E.cand.push_back(TuneCand{TM_LPT, max_grid});
        E.cand.push_back(TuneCand{TM_LPT, std::max(256, max_grid / 4)});
        if (xcd_ok) {
            E.cand.push_back(TuneCand{TM_STATIC, max_grid});
            E.cand.push_back(TuneCand{TM_XLPT, max_grid});
        }
    }
    tune_poll(T, E);
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(s, &cst) == hipSuccess && cst != hipStreamCaptureStatusNone;
    // a captured launch keeps its counter slot for every replay, so graphs take
    // no queue mapping (the slots rotate over later eager launches)
    if (E.best >= 0) {
        const TuneCand& B = E.cand[E.best];
        if (capturing && (B.mode == TM_LPT || B.mode == TM_XLPT)) return fixed;
        return TileChoice{B.mode, B.grid, -1};
    }
    if (capturing) return fixed;
    const int c = E.next++ % (int)E.cand.size();
    return TileChoice{E.cand[c].mode, E.cand[c].grid, c};
}

void tile_sample(const char* name, int cand, hipEvent_t e0, hipEvent_t e1, int64_t tiles) {
    Tuner& T = tuner();
    std::lock_guard<std::mutex> lk(T.mu);
    T.table[name].pending.push_back(TuneEntry::Pending{cand, e0, e1, tiles});
}

hipEvent_t Meter::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    DD_HIP(hipEventCreate(&e));
    return e;
}
}  // namespace dd

extern "C" {

int dd_autotune_report(char* buf, int64_t len) {
    DD_GUARD_BEGIN
    Tuner& T = tuner();
    std::lock_guard<std::mutex> lk(T.mu);
    std::string out;
    static const char* mname[4] = {"static", "xcd", "lpt-queue", "xcd-lpt-queue"};
    std::vector<std::string> names;
    for (auto& kv : T.table) names.push_back(kv.first);
    std::sort(names.begin(), names.end());
    for (const auto& nm : names) {
        TuneEntry& E = T.table[nm];
        tune_poll(T, E);
        out += nm + ":";
        for (size_t c = 0; c < E.cand.size(); ++c) {
            const TuneCand& C = E.cand[c];
            char tmp[160];
            std::snprintf(tmp, sizeof tmp, " %s%s/%d=%.3gus/tile(%d)", (int)c == E.best ? "*" : "", mname[C.mode],
                          C.grid, C.tiles > 0 ? 1e3 * C.ms / C.tiles : 0.0, C.n);
            out += tmp;
        }
        out += "\n";
    }
    if (buf && len > 0) {
        const size_t k = std::min<size_t>(out.size(), (size_t)len - 1);
        std::memcpy(buf, out.data(), k);
        buf[k] = 0;
    }
    return (int)std::min<size_t>(out.size(), (size_t)INT32_MAX);
    DD_GUARD_END
}

int dd_meter_start(const char* kernel) {
    DD_GUARD_BEGIN
    Meter& m = meter();
    for (hipEvent_t e : m.ev) m.pool.push_back(e);
    m.ev.clear();
    m.flops = m.bytes = 0.0;
    m.launches = 0;
    m.name = kernel ? kernel : "";
    return DD_OK;
    DD_GUARD_END
}

int dd_meter_read(dd_meter_t* out) {
    if (!out) return DD_ERR_INVALID_ARG;
    DD_GUARD_BEGIN
    Meter& m = meter();
    double ms = 0.0;
    if (!m.ev.empty()) DD_HIP(hipEventSynchronize(m.ev.back()));
    for (size_t k = 0; k + 1 < m.ev.size(); k += 2) {
        float t = 0.f;
        DD_HIP(hipEventElapsedTime(&t, m.ev[k], m.ev[k + 1]));
        ms += t;
    }
    out->launches = m.launches;
    out->total_ms = ms;
    out->flops = m.flops;
    out->bytes = m.bytes;
    return DD_OK;
    DD_GUARD_END
}

int dd_trim_device_cache(void) {
    DD_GUARD_BEGIN
    DeviceCache& c = device_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    std::vector<int> devs;
    for (auto& kv : c.free_) devs.push_back(kv.first.first);
    std::sort(devs.begin(), devs.end());
    devs.erase(std::unique(devs.begin(), devs.end()), devs.end());
    for (int d : devs) trim_locked(c, d);
    return DD_OK;
    DD_GUARD_END
}

const char* dd_strerror(int code) {
    switch (code) {
        case DD_OK: return "ok";
        case DD_ERR_INVALID_ARG: return "invalid argument";
        case DD_ERR_NOT_SPD: return "matrix (local block or coarse operator) is not SPD";
        case DD_ERR_EIG: return "local eigen/polar iteration failed";
        case DD_ERR_NAN: return "NaN or Inf encountered";
        case DD_ERR_OOM: return "out of device memory";
        case DD_ERR_HIP: return "HIP runtime error";
        case DD_ERR_INTERNAL: return "internal error";
        case DD_WARN_MAXIT: return "PCG reached maxit";
        case DD_WARN_FULL_COARSE: return "tau >= 1: every local mode kept (coarse space = whole space)";
        case DD_WARN_FP32_FALLBACK: return "FP32 local factor fell back to FP64";
        default: return "unknown";
    }
}

const char* dd_phase_name(int32_t phase) {
    if (phase < 0 || phase >= DD_NPHASE) return "?";
    return kPhaseNames[phase];
}

int dd_partition_ggg(const dd_csr* A, int32_t N, uint64_t seed, int32_t* part, hipStream_t stream) {
    DD_GUARD_BEGIN
    if (!A || !part || A->n <= 0 || N < 1 || N > A->n) return DD_ERR_INVALID_ARG;
    CsrDev C{A->n, A->nnz, A->rowptr, A->colind, A->val};
    ggg_partition(C, N, seed, part, stream);
    return DD_OK;
    DD_GUARD_END
}

int dd_partition_ggg_noalloc(const dd_csr* A, int32_t N, uint64_t seed, int32_t* part, hipStream_t stream) {
    DD_GUARD_BEGIN
    if (!A || !part || A->n <= 0 || N < 1 || N > A->n) return DD_ERR_INVALID_ARG;
    if (A->n > kGggMaxN || N > kGggMaxParts) return DD_ERR_INVALID_ARG;
    CsrDev C{A->n, A->nnz, A->rowptr, A->colind, A->val};
    ggg_partition_noalloc(C, N, seed, part, stream);
    return DD_OK;
    DD_GUARD_END
}

__global__ void k_check_finite(const double* v, int64_t n, int32_t* bad) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(v[i])) atomicOr(bad, 1);
}

// The CSR structure dd_setup assumes (full symmetric storage): rowptr[0] = 0,
// rowptr[n] = nnz, rows non-decreasing, column indices in [0, n) and strictly
// increasing within each row, and (j, i) stored whenever (i, j) is (binary
// search of row j).  Every read is checked first, so a malformed input only
// sets the flag.
__global__ void k_check_pattern(const int32_t* rowptr, const int32_t* colind, int64_t n, int64_t nnz, int32_t* bad) {
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t0 == 0 && (rowptr[0] != 0 || rowptr[n] != nnz)) atomicOr(bad, 1);
    for (int64_t i = t0; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = rowptr[i], e = rowptr[i + 1];
        if (b < 0 || e < b || e > nnz) {
            atomicOr(bad, 1);
            continue;
        }
        int64_t prev = -1;
        for (int64_t k = b; k < e; ++k) {
            const int64_t j = colind[k];
            if (j < 0 || j >= n || j <= prev) {
                atomicOr(bad, 1);
                break;
            }
            prev = j;
            int64_t lo = rowptr[j], hi = (int64_t)rowptr[j + 1] - 1;
            if (lo < 0 || hi >= nnz) {
                atomicOr(bad, 1);
                break;
            }
            bool found = false;
            while (lo <= hi) {
                const int64_t mid = (lo + hi) >> 1;
                const int64_t c = colind[mid];
                if (c == i) { found = true; break; }
                if (c < i) lo = mid + 1;
                else hi = mid - 1;
            }
            if (!found) {
                atomicOr(bad, 1);
                break;
            }
        }
    }
}

}  // extern "C"

namespace dd {
// Level 0 from device CSR arrays and a partition (copied), then every level of
// the hierarchy (R8) and the diagnostics.  Returns DD_OK, a warning, or an
// error with H unusable.
static int build_handle(Handle& H, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                        const double* val, const int32_t* part, int32_t N, int32_t overlap, double tau, int32_t levels,
                        hipStream_t s) {
    H.levels_req = levels;
    auto lv = std::make_unique<Level>();
    Level& L0 = *lv;
    L0.n = n;
    L0.nnz = nnz;
    L0.rowptr.alloc(n + 1);
    L0.colind.alloc(nnz);
    L0.val.alloc(nnz);
    DD_HIP(hipMemcpyAsync(L0.rowptr.p, rowptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    DD_HIP(hipMemcpyAsync(L0.colind.p, colind, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    DD_HIP(hipMemcpyAsync(L0.val.p, val, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    {
        DBuf<int32_t> bad(1);
        DD_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, s, L0.val.p, L0.nnz, bad.p);
        int32_t hb = 0;
        DD_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DD_HIP(hipStreamSynchronize(s));
        if (hb) return DD_ERR_NAN;
        if (H.opt.validate) {
            DD_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
            hipLaunchKernelGGL(k_check_pattern, dim3(vgrid(n)), dim3(256), 0, s, L0.rowptr.p, L0.colind.p, n, nnz,
                               bad.p);
            launch_check("check_pattern");
            DD_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DD_HIP(hipStreamSynchronize(s));
            if (hb) return DD_ERR_INVALID_ARG;
        }
    }
    L0.N = N;
    L0.delta = overlap;
    L0.tau = tau;
    L0.part.alloc(n);
    DD_HIP(hipMemcpyAsync(L0.part.p, part, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    L0.hsub = H.sub_off;  // empty unless a batch
    {
        DBuf<int32_t> cnt(N);
        const int rc = validate_partition(L0.part.p, n, N, cnt.p, s);
        if (rc != DD_OK) return rc;
    }
    H.lv.push_back(std::move(lv));
    // levels - 1 decomposed levels; the coarse operator of the last one is
    // factored, the others hand E to the next level (R8)
    for (int l = 0; l + 1 < levels; ++l) {
        Level& Lv = *H.lv[l];
        const bool more = l + 2 < levels;
        std::unique_ptr<Level> nx = more ? std::make_unique<Level>() : nullptr;
        build_level(Lv, H.opt, H.info, s, more ? nx.get() : nullptr);
        if (!more || Lv.nC == 0) break;
        partition_next(Lv, *nx, H.opt.coarsen, s);
        H.lv.push_back(std::move(nx));
    }
    for (auto& l : H.lv) alloc_krylov(*l, H.opt.schwarz == DD_SCHWARZ_DEFLATED);
    // diagnostics
    dd_info_t& I = H.info;
    I.levels = (int32_t)H.lv.size() + 1;
    double gsum = 0.0;
    for (size_t l = 0; l < H.lv.size(); ++l) {
        I.N[l] = H.lv[l]->N;
        I.n[l] = H.lv[l]->n;
        gsum += (double)H.lv[l]->n;
    }
    I.n[H.lv.size()] = H.lv.back()->nC;
    gsum += (double)H.lv.back()->nC;
    I.n_C = L0.nC;
    I.grid_complexity = gsum / double(n);
    I.p_min = N ? *std::min_element(L0.p.begin(), L0.p.end()) : 0;
    I.p_max = N ? *std::max_element(L0.p.begin(), L0.p.end()) : 0;
    for (int b = 0; b < DD_PHIST; ++b) I.p_hist[b] = 0;
    for (int i = 0; i < N; ++i) {
        int b = 0;
        while (b + 1 < DD_PHIST && L0.p[i] >= (1 << b)) ++b;
        I.p_hist[b] += 1;
    }
    I.k_c = 0;  // computed at the first dd_info call
    I.eig_iters_max = 0;
    I.eig_iters_mean = 0.0;
    I.eig_resid_max = 0.0;
    if ((int)L0.lob_iters.size() == N && N > 0) {
        double sum = 0.0;
        for (int i = 0; i < N; ++i) {
            I.eig_iters_max = std::max(I.eig_iters_max, L0.lob_iters[i]);
            sum += L0.lob_iters[i];
            I.eig_resid_max = std::max(I.eig_resid_max, L0.lob_resid[i]);
        }
        I.eig_iters_mean = sum / N;
    }
    if (!H.partial.p) {
        const int w = std::max(64, H.nsys());
        H.partial.alloc((int64_t)512 * w);
        H.dots.alloc(w);
        DD_HIP(hipHostMalloc(&H.hpin, w * sizeof(double)));
    }
    int64_t bytes = 0;
    for (auto& l : H.lv)
        bytes += l->W.buf.bytes() + l->W32.buf.bytes() + l->Z.buf.bytes() + l->E.bytes() + l->memb.bytes() + l->ext.bytes();
    I.device_bytes = bytes;
    I.coarse_factor_bytes = H.lv.empty() ? 0 : H.lv.back()->E.bytes();
    if (tau >= 1.0) return DD_WARN_FULL_COARSE;
    return I.fp32_fallbacks > 0 ? DD_WARN_FP32_FALLBACK : DD_OK;
}
}  // namespace dd

extern "C" {

int dd_setup(const dd_csr* A, const int32_t* part, int32_t N, int32_t overlap, double tau, int32_t levels,
             const dd_options* opt, hipStream_t s, dd_handle* out) {
    DD_GUARD_BEGIN
    if (!A || !part || !out) return DD_ERR_INVALID_ARG;
    *out = nullptr;
    if (A->n <= 0 || A->nnz <= 0 || N < 1 || N > A->n || overlap < 1 || overlap > 200 || !(tau > 0.0) || levels < 2 ||
        levels > DD_MAX_LEVELS)
        return DD_ERR_INVALID_ARG;
    auto hd = std::make_unique<dd_handle_s>();
    Handle& H = hd->h;
    if (parse_opts(opt, H.opt) != DD_OK) return DD_ERR_INVALID_ARG;
    const int rc = build_handle(H, A->n, A->nnz, A->rowptr, A->colind, A->val, part, N, overlap, tau, levels, s);
    if (rc < 0) return rc;
    *out = hd.release();
    return rc;
    DD_GUARD_END
}

int dd_extract_local(const dd_csr* A, const int32_t* part, int32_t N, int32_t overlap, int32_t i, int32_t* sizes,
                     double* Aii, double* X, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!A || !part || A->n <= 0 || A->nnz <= 0 || N < 1 || N > A->n || overlap < 1 || overlap > 200 || i < 0 ||
        i >= N)
        return DD_ERR_INVALID_ARG;
    Level L;
    L.n = A->n;
    L.nnz = A->nnz;
    L.rowptr.alloc(L.n + 1);
    L.colind.alloc(L.nnz);
    L.val.alloc(L.nnz);
    DD_HIP(hipMemcpyAsync(L.rowptr.p, A->rowptr, (L.n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    DD_HIP(hipMemcpyAsync(L.colind.p, A->colind, L.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    DD_HIP(hipMemcpyAsync(L.val.p, A->val, L.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    L.N = N;
    L.delta = overlap;
    L.part.alloc(L.n);
    DD_HIP(hipMemcpyAsync(L.part.p, part, L.n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    {
        DBuf<int32_t> cnt(N);
        const int rc = validate_partition(L.part.p, L.n, N, cnt.p, s);
        if (rc != DD_OK) return rc;
    }
    dd_info_t info{};
    Timer tm(s);
    Arena Y;
    sets_and_extract(L, info, tm, Y, s);
    const int ni = L.ni[i], nt = L.nt[i];
    if (sizes) {
        sizes[0] = L.nI[i];
        sizes[1] = L.nG[i];
        sizes[2] = L.nD[i];
    }
    if (Aii) {
        d2h(Aii, L.L.ptr[i], (size_t)ni * ni, s);
        DD_HIP(hipStreamSynchronize(s));
    }
    if (X) {  // Y_i = X_i^T is n~_i x n_i, column-major: X_i(r, c) = Y_i(c, r)
        const auto y = to_host(Y.ptr[i], (size_t)nt * ni, s);
        for (int r = 0; r < ni; ++r)
            for (int c = 0; c < nt; ++c) X[r + (int64_t)c * ni] = y[c + (int64_t)r * nt];
    }
    return DD_OK;
    DD_GUARD_END
}

int dd_update_values(dd_handle h, const double* val, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!h || !val || h->h.lv.empty()) return DD_ERR_INVALID_ARG;
    const Level& L0 = *h->h.lv[0];
    // the new hierarchy is built beside the old one and replaces it only on success
    auto fresh = std::make_unique<dd_handle_s>();
    Handle& F = fresh->h;
    F.opt = h->h.opt;
    // a batch handle: the systems' subdomain ranges, so that every level is
    // partitioned system by system again (the dof ranges stay with the handle)
    F.sub_off = h->h.sub_off;
    F.sys_off = h->h.sys_off;
    const int rc = build_handle(F, L0.n, L0.nnz, L0.rowptr.p, L0.colind.p, val, L0.part.p, L0.N, L0.delta, L0.tau,
                                h->h.levels_req, s);
    if (rc < 0) return rc;
    DD_HIP(hipStreamSynchronize(s));
    std::swap(h->h.lv, F.lv);
    h->h.info = F.info;
    // the captured PCG graph and the block state point into the old levels'
    // buffers, which go with F: both are rebuilt on next use
    h->h.gp.reset();
    h->h.bp.reset();
    return rc;
    DD_GUARD_END
}

int dd_setup_batch(const dd_csr* As, const int32_t* const* parts, const int32_t* Ns, int32_t nsys, int32_t overlap,
                   double tau, int32_t levels, const dd_options* opt, hipStream_t s, dd_handle* out) {
    DD_GUARD_BEGIN
    if (!As || !parts || !Ns || !out || nsys < 1) return DD_ERR_INVALID_ARG;
    *out = nullptr;
    if (overlap < 1 || overlap > 200 || !(tau > 0.0) || levels < 2 || levels > DD_MAX_LEVELS) return DD_ERR_INVALID_ARG;
    std::vector<int64_t> noff(nsys + 1, 0), zoff(nsys + 1, 0), poff(nsys + 1, 0);
    for (int j = 0; j < nsys; ++j) {
        const dd_csr& A = As[j];
        if (A.n <= 0 || A.nnz <= 0 || !A.rowptr || !A.colind || !A.val || !parts[j] || Ns[j] < 1 || Ns[j] > A.n)
            return DD_ERR_INVALID_ARG;
        noff[j + 1] = noff[j] + A.n;
        zoff[j + 1] = zoff[j] + A.nnz;
        poff[j + 1] = poff[j] + Ns[j];
    }
    if (noff[nsys] >= ((int64_t)1 << 31) || zoff[nsys] >= ((int64_t)1 << 31) || poff[nsys] > noff[nsys])
        return DD_ERR_INVALID_ARG;
    auto hd = std::make_unique<dd_handle_s>();
    Handle& H = hd->h;
    if (parse_opts(opt, H.opt) != DD_OK) return DD_ERR_INVALID_ARG;
    // the deflated variant needs GMRES, which has no per-system form: refused for a batch
    if (H.opt.schwarz != DD_SCHWARZ_ADDITIVE) return DD_ERR_INVALID_ARG;
    // every system's own CSR structure is checked before the union shifts its
    // indices (an out-of-range column must not land inside another system)
    if (H.opt.validate) {
        DBuf<int32_t> bad(1);
        for (int j = 0; j < nsys; ++j) {
            DD_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
            hipLaunchKernelGGL(k_check_pattern, dim3(vgrid(As[j].n)), dim3(256), 0, s, As[j].rowptr, As[j].colind,
                               As[j].n, As[j].nnz, bad.p);
            launch_check("check_pattern");
            int32_t hb = 0;
            DD_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DD_HIP(hipStreamSynchronize(s));
            if (hb) return DD_ERR_INVALID_ARG;
        }
    }
    // the block-diagonal union of the systems, its partition and the system of every dof
    const int64_t n = noff[nsys], nnz = zoff[nsys];
    DBuf<int32_t> rowptr(n + 1), colind(nnz), part(n);
    DBuf<double> val(nnz);
    H.sys_id.alloc(n);
    for (int j = 0; j < nsys; ++j) {
        const dd_csr& A = As[j];
        const int g1 = vgrid(A.n + 1), g2 = vgrid(A.nnz);
        hipLaunchKernelGGL(k_copy_add_i32, dim3(g1), dim3(256), 0, s, A.rowptr, rowptr.p + noff[j], A.n + 1, zoff[j]);
        hipLaunchKernelGGL(k_copy_add_i32, dim3(g2), dim3(256), 0, s, A.colind, colind.p + zoff[j], A.nnz, noff[j]);
        hipLaunchKernelGGL(k_copy_add_i32, dim3(g1), dim3(256), 0, s, parts[j], part.p + noff[j], A.n, poff[j]);
        hipLaunchKernelGGL(k_set_i32, dim3(g1), dim3(256), 0, s, H.sys_id.p + noff[j], A.n, j);
        DD_HIP(hipMemcpyAsync(val.p + zoff[j], A.val, A.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
        launch_check("batch_union");
    }
    H.sys_off = noff;
    H.dsys_off = upload(noff, s);
    H.sub_off.assign(poff.begin(), poff.end());
    H.dscal.alloc(2 * nsys);
    DD_HIP(hipHostMalloc(&H.hscal, 2 * nsys * sizeof(double)));
    const int rc = build_handle(H, n, nnz, rowptr.p, colind.p, val.p, part.p, (int32_t)poff[nsys], overlap, tau,
                                levels, s);
    if (rc < 0) return rc;
    DD_HIP(hipStreamSynchronize(s));
    *out = hd.release();
    return rc;
    DD_GUARD_END
}

// ---------------------------------------------------------------------------
// warm-start network
// ---------------------------------------------------------------------------
struct dd_model_s {
    Model m;
};

static Level* level_of(dd_handle h, int32_t level) {
    if (!h || level < 0 || level >= (int)h->h.lv.size()) return nullptr;
    return h->h.lv[level].get();
}

int dd_model_create(uint64_t seed, dd_model* out) {
    DD_GUARD_BEGIN
    if (!out) return DD_ERR_INVALID_ARG;
    *out = nullptr;
    auto md = std::make_unique<dd_model_s>();
    // Glorot-scaled normal weights from a SplitMix64 stream (Box-Muller),
    // zero biases, output bias softplus^{-1}(1) so that every weight starts at 1
    std::vector<double> p(WS_P, 0.0);
    uint64_t k = 0;
    auto draw = [&]() {
        auto mix = [&](uint64_t c) {
            uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            return z ^ (z >> 31);
        };
        const double u1 = ((mix(k) >> 11) + 1.0) * 0x1.0p-53, u2 = (mix(k + 1) >> 11) * 0x1.0p-53;
        k += 2;
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    };
    int o = 0;
    for (int i = 0; i < WS_H * WS_F; ++i) p[o++] = draw() * std::sqrt(1.0 / WS_F);
    o += WS_H;
    for (int i = 0; i < WS_H * WS_H; ++i) p[o++] = draw() * std::sqrt(1.0 / WS_H);
    o += WS_H;
    for (int i = 0; i < WS_H; ++i) p[o++] = draw() * std::sqrt(1.0 / WS_H) * 0.1;
    p[o] = std::log(std::exp(1.0) - 1.0);
    Model& M = md->m;
    h2d(M.params.p, p.data(), WS_P, nullptr);
    std::vector<double> zero(WS_P, 0.0), one(WS_F, 1.0);
    h2d(M.m1.p, zero.data(), WS_P, nullptr);
    h2d(M.m2.p, zero.data(), WS_P, nullptr);
    h2d(M.mean.p, zero.data(), WS_F, nullptr);
    h2d(M.stdv.p, one.data(), WS_F, nullptr);
    DD_HIP(hipStreamSynchronize(nullptr));
    *out = md.release();
    return DD_OK;
    DD_GUARD_END
}

void dd_model_destroy(dd_model m) { delete m; }

int dd_model_add_samples(dd_model md, dd_handle h, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!md || !h || h->h.lv.empty()) return DD_ERR_INVALID_ARG;
    Level& Lv = *h->h.lv[0];
    if (!Lv.Tb32.h.empty() || !Lv.W.buf.p) return DD_ERR_INVALID_ARG;  // needs the FP64 local inverses
    Model& M = md->m;
    const int N = Lv.N;
    const auto& ni = Lv.ni;
    const auto& nI = Lv.nI;
    const auto& nD = Lv.nD;
    std::vector<int> act(N);
    std::vector<int64_t> hoffD(N + 1, 0);
    int nsub = 0;
    for (int i = 0; i < N; ++i) {
        if (Lv.p[i] > JAC_MAX) return DD_ERR_INVALID_ARG;  // the basis of the target needs p_i <= 128
        act[i] = Lv.p[i] > 0 && nD[i] > 0;
        hoffD[i + 1] = hoffD[i] + (act[i] ? nD[i] : 0);
        nsub += act[i];
    }
    const int64_t tot = hoffD[N];
    if (!tot) return DD_OK;
    // U_i = A_ii^{-1} [Z_i; 0] = W_i^T W_i [Z_i; 0]
    Arena U0, U1, Gt, Q;
    std::vector<int64_t> su(N), sg(N);
    for (int i = 0; i < N; ++i) {
        su[i] = act[i] ? (int64_t)ni[i] * Lv.p[i] : 1;
        sg[i] = act[i] ? (int64_t)nD[i] * Lv.p[i] : 1;
    }
    U0.alloc(su); U1.alloc(su); Gt.alloc(sg); Q.alloc(sg);
    fill(U0.buf.p, U0.buf.n, 0.0, s);
    {
        std::vector<double*> zp(Lv.Z.ptr.begin(), Lv.Z.ptr.end());
        Batch<DMat> Zs = mats(zp, nI, nI, Lv.p, s, &act), Zd = mats(U0.ptr, ni, nI, Lv.p, s, &act);
        copy_vb(Zs, Zd, false, 1.0, s);
        Batch<GemmItem> g1, g2;
        for (int i = 0; i < N; ++i) {
            if (!act[i]) continue;
            g1.h.push_back(GemmItem{Lv.W.ptr[i], ni[i], U0.ptr[i], ni[i], U1.ptr[i], ni[i], ni[i], Lv.p[i], ni[i], 1.0, 0.0});
            g2.h.push_back(GemmItem{Lv.W.ptr[i], ni[i], U1.ptr[i], ni[i], U0.ptr[i], ni[i], ni[i], Lv.p[i], ni[i], 1.0, 0.0});
        }
        g1.sync(s);
        g2.sync(s);
        gemm_vb(g1, false, false, s);
        gemm_vb(g2, true, false, s);
    }
    // Gt_i = A(Delta_i, Omega_i) U_i; target^2 = (row leverage of orth(Gt_i)) * |Delta_i| / p_i
    DBuf<int64_t> offD = upload(hoffD, s);
    std::vector<int32_t> pc(N);
    for (int i = 0; i < N; ++i) pc[i] = act[i] ? Lv.p[i] : 0;
    DBuf<int32_t> dpc = upload(pc, s);
    DBuf<double*> dU(N), dG(N);
    h2d(dU.p, U0.ptr.data(), N, s);
    h2d(dG.p, Gt.ptr.data(), N, s);
    // a level's own offsets of Delta (all subdomains) are needed by the kernel: inactive ones have 0 rows
    const WsMaps WM = ws_maps(Lv);
    {
        // the kernel walks rows offD[i] .. offD[i+1] of subdomain i; for an inactive
        // subdomain that range is empty, so its Delta count in the maps is never used
        ws_adjoint_product(WM, offD.p, tot, dU.p, dG.p, dpc.p, s);
    }
    std::vector<OrthItem> oi;
    for (int i = 0; i < N; ++i)
        if (act[i]) oi.push_back(OrthItem{Gt.ptr[i], nD[i], Lv.p[i], Q.ptr[i]});
    orth_basis_vb(oi, s);
    DBuf<double> lev(tot), feats((size_t)tot * WS_F), smean(N);
    {
        Batch<RowItem> rb;
        for (int i = 0; i < N; ++i)
            if (act[i])
                rb.h.push_back(RowItem{Q.ptr[i], nD[i], nD[i], Lv.p[i], lev.p + hoffD[i], (double)nD[i] / Lv.p[i]});
        rb.sync(s);
        ws_row_leverage(rb, s);
    }
    ws_subdomain_logdiag(WM, smean.p, s);
    ws_features(WM, smean.p, offD.p, tot, feats.p, s);
    auto hl = to_host(lev.p, tot, s);
    std::vector<double> ht(tot), hw(tot);
    for (int i = 0; i < N; ++i)
        for (int64_t e = hoffD[i]; e < hoffD[i + 1]; ++e) {
            ht[e] = std::sqrt(std::max(0.0, hl[e]));
            hw[e] = 1.0 / (double)(hoffD[i + 1] - hoffD[i]);
        }
    // append to the store
    const int64_t n0 = M.ns, n1 = n0 + tot;
    auto grow = [&](DBuf<double>& b, int64_t per) {
        DBuf<double> nb((size_t)n1 * per);
        if (n0) DD_HIP(hipMemcpyAsync(nb.p, b.p, (size_t)n0 * per * sizeof(double), hipMemcpyDeviceToDevice, s));
        DD_HIP(hipStreamSynchronize(s));
        b = std::move(nb);
    };
    grow(M.feats, WS_F);
    grow(M.target, 1);
    grow(M.weight, 1);
    DD_HIP(hipMemcpyAsync(M.feats.p + n0 * WS_F, feats.p, (size_t)tot * WS_F * sizeof(double), hipMemcpyDeviceToDevice, s));
    h2d(M.target.p + n0, ht.data(), tot, s);
    h2d(M.weight.p + n0, hw.data(), tot, s);
    DD_HIP(hipStreamSynchronize(s));
    M.ns = n1;
    M.nsub += nsub;
    return DD_OK;
    DD_GUARD_END
}

int dd_model_train(dd_model md, int32_t epochs, double lr, double* loss, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!md || epochs < 0 || !(lr > 0.0)) return DD_ERR_INVALID_ARG;
    Model& M = md->m;
    if (M.ns == 0) return DD_ERR_INVALID_ARG;
    if (!M.stats) {
        ws_feature_stats(M.feats.p, M.ns, M.mean.p, M.stdv.p, s);
        M.stats = true;
    }
    const double scale = 1.0 / std::max(1, M.nsub);  // mean over subdomains of each one's mean square error
    for (int e = 0; e < epochs; ++e) {
        mlp_loss_grad(M.params.p, M.mean.p, M.stdv.p, M.feats.p, M.target.p, M.weight.p, M.ns, M.grad.p, M.dloss.p, s);
        mlp_adam(M.params.p, M.grad.p, M.m1.p, M.m2.p, lr, ++M.step, s);
        if (loss) {
            double l = 0.0;
            d2h(&l, M.dloss.p, 1, s);
            DD_HIP(hipStreamSynchronize(s));
            loss[e] = l * scale;
        }
    }
    DD_HIP(hipStreamSynchronize(s));
    return DD_OK;
    DD_GUARD_END
}

int dd_model_params(dd_model md, double* out, int32_t* count) {
    DD_GUARD_BEGIN
    if (!md) return DD_ERR_INVALID_ARG;
    if (count) *count = WS_P + 2 * WS_F;
    if (out) {
        d2h(out, md->m.params.p, WS_P, nullptr);
        d2h(out + WS_P, md->m.mean.p, WS_F, nullptr);
        d2h(out + WS_P + WS_F, md->m.stdv.p, WS_F, nullptr);
        DD_HIP(hipStreamSynchronize(nullptr));
    }
    return DD_OK;
    DD_GUARD_END
}

int dd_model_set_params(dd_model md, const double* in, int32_t count) {
    DD_GUARD_BEGIN
    if (!md || !in || count != WS_P + 2 * WS_F) return DD_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        if (!std::isfinite(in[i])) return DD_ERR_NAN;
    for (int f = 0; f < WS_F; ++f)
        if (!(in[WS_P + WS_F + f] > 0.0)) return DD_ERR_INVALID_ARG;
    h2d(md->m.params.p, in, WS_P, nullptr);
    h2d(md->m.mean.p, in + WS_P, WS_F, nullptr);
    h2d(md->m.stdv.p, in + WS_P + WS_F, WS_F, nullptr);
    DD_HIP(hipStreamSynchronize(nullptr));
    md->m.stats = true;
    return DD_OK;
    DD_GUARD_END
}

int dd_model_forward(dd_model md, const double* feats, int64_t n, double* out, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!md || n < 0 || (n > 0 && (!feats || !out))) return DD_ERR_INVALID_ARG;
    mlp_forward(md->m.params.p, md->m.mean.p, md->m.stdv.p, feats, n, out, s);
    return DD_OK;
    DD_GUARD_END
}

int dd_model_loss_grad(dd_model md, const double* feats, const double* target, const double* weight, int64_t n,
                       double* loss, double* grad, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!md || n < 1 || !feats || !target || !weight) return DD_ERR_INVALID_ARG;
    Model& M = md->m;
    mlp_loss_grad(M.params.p, M.mean.p, M.stdv.p, feats, target, weight, n, M.grad.p, M.dloss.p, s);
    if (loss) d2h(loss, M.dloss.p, 1, s);
    if (grad) d2h(grad, M.grad.p, WS_P, s);
    DD_HIP(hipStreamSynchronize(s));
    return DD_OK;
    DD_GUARD_END
}

int dd_model_samples(dd_model md, int64_t* n, double* feats, double* target, double* weight) {
    DD_GUARD_BEGIN
    if (!md) return DD_ERR_INVALID_ARG;
    const Model& M = md->m;
    if (n) *n = M.ns;
    if (feats) d2h(feats, M.feats.p, (size_t)M.ns * WS_F, nullptr);
    if (target) d2h(target, M.target.p, M.ns, nullptr);
    if (weight) d2h(weight, M.weight.p, M.ns, nullptr);
    DD_HIP(hipStreamSynchronize(nullptr));
    return DD_OK;
    DD_GUARD_END
}

int dd_subdomain_eig_stats(dd_handle h, int32_t level, int32_t* iters, double* resid) {
    Level* L = level_of(h, level);
    if (!L) return DD_ERR_INVALID_ARG;
    if ((int)L->lob_iters.size() != L->N) return DD_ERR_INVALID_ARG;  // dense route: no iterations
    if (iters) std::copy(L->lob_iters.begin(), L->lob_iters.end(), iters);
    if (resid) std::copy(L->lob_resid.begin(), L->lob_resid.end(), resid);
    return DD_OK;
}

int dd_apply(dd_handle h, const double* r, double* z, int32_t nrhs, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!h || !r || !z || nrhs < 1) return DD_ERR_INVALID_ARG;
    const int64_t n = h->h.lv[0]->n;
    if (nrhs > 1 && block_ok(h->h)) {
        for (int k0 = 0; k0 < nrhs; k0 += kMrhs)
            apply_block(h->h, r + (int64_t)k0 * n, z + (int64_t)k0 * n, std::min(kMrhs, nrhs - k0), s);
    } else {
        for (int k = 0; k < nrhs; ++k) apply_level(h->h, 0, r + (int64_t)k * n, z + (int64_t)k * n, s);
    }
    return DD_OK;
    DD_GUARD_END
}

int dd_pcg(dd_handle h, const double* b, double* x, int32_t nrhs, double rtol, int32_t maxit, int32_t* iters,
           double* relres, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!h || !b || !x || nrhs < 1 || maxit < 0 || !(rtol > 0.0)) return DD_ERR_INVALID_ARG;
    Handle& H = h->h;
    if (H.opt.schwarz == DD_SCHWARZ_DEFLATED) return DD_ERR_INVALID_ARG;  // not symmetric: dd_gmres
    const int64_t n = H.lv[0]->n;
    int rc = DD_OK;
    if (H.nsys() > 1) {  // batch: one PCG per system, nsys results per right-hand side
        const int ns = H.nsys();
        std::vector<int> it(ns);
        std::vector<double> rr(ns);
        const bool graph = H.opt.graph_pcg > 0 && H.lv.size() == 1 && H.opt.schwarz == DD_SCHWARZ_ADDITIVE;
        for (int k = 0; k < nrhs; ++k) {
            const int c = graph ? krylov_graph_seg(H, b + k * n, x + k * n, rtol, maxit, it.data(), rr.data(), s)
                                : krylov_seg(H, 0, b + k * n, x + k * n, rtol, maxit, H.lv.size() > 1, true,
                                             it.data(), rr.data(), s);
            if (c < 0) return c;
            if (c > 0) rc = c;
            for (int j = 0; j < ns; ++j) {
                if (iters) iters[(int64_t)k * ns + j] = it[j];
                if (relres) relres[(int64_t)k * ns + j] = rr[j];
            }
            if (k == 0) {
                H.info.last_iters = *std::max_element(it.begin(), it.end());
                H.info.last_relres = *std::max_element(rr.begin(), rr.end());
            }
        }
        return rc;
    }
    if (nrhs > 1 && block_ok(H)) {
        std::vector<int> it(kMrhs);
        std::vector<double> rr(kMrhs);
        for (int k0 = 0; k0 < nrhs; k0 += kMrhs) {
            const int K = std::min(kMrhs, nrhs - k0);
            const int c = krylov_block(H, b + k0 * n, x + k0 * n, K, rtol, maxit, it.data(), rr.data(), s);
            if (c < 0) return c;
            if (c > 0) rc = c;
            for (int k = 0; k < K; ++k) {
                if (iters) iters[k0 + k] = it[k];
                if (relres) relres[k0 + k] = rr[k];
            }
            if (k0 == 0) {
                H.info.last_iters = it[0];
                H.info.last_relres = rr[0];
            }
        }
        return rc;
    }
    const bool graph = H.opt.graph_pcg > 0 && H.lv.size() == 1 && H.opt.schwarz == DD_SCHWARZ_ADDITIVE;
    for (int k = 0; k < nrhs; ++k) {
        int it = 0;
        double rr = 0.0;
        const int c = graph ? krylov_graph(H, b + k * n, x + k * n, rtol, maxit, &it, &rr, s)
                            : krylov(H, 0, b + k * n, x + k * n, rtol, maxit, H.lv.size() > 1, true, &it, &rr, s);
        if (c < 0) return c;
        if (c > 0) rc = c;
        if (iters) iters[k] = it;
        if (relres) relres[k] = rr;
        if (k == 0) {
            H.info.last_iters = it;
            H.info.last_relres = rr;
        }
    }
    return rc;
    DD_GUARD_END
}

int dd_gmres(dd_handle h, const double* b, double* x, int32_t nrhs, double rtol, int32_t maxit, int32_t restart,
             int32_t* iters, double* relres, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!h || !b || !x || nrhs < 1 || maxit < 0 || !(rtol > 0.0) || restart < 1 || restart > kMaxRestart)
        return DD_ERR_INVALID_ARG;
    Handle& H = h->h;
    if (H.nsys() > 1) return DD_ERR_INVALID_ARG;  // batch handles: one PCG per system (dd_pcg)
    const int64_t n = H.lv[0]->n;
    int rc = DD_OK;
    for (int k = 0; k < nrhs; ++k) {
        int it = 0;
        double rr = 0.0;
        const int c = gmres(H, 0, b + k * n, x + k * n, rtol, maxit, restart, &it, &rr, s);
        if (c < 0) return c;
        if (c > 0) rc = c;
        if (iters) iters[k] = it;
        if (relres) relres[k] = rr;
        if (k == 0) {
            H.info.last_iters = it;
            H.info.last_relres = rr;
        }
    }
    return rc;
    DD_GUARD_END
}

int dd_spmv(dd_handle h, const double* x, double* y, hipStream_t s) {
    DD_GUARD_BEGIN
    if (!h || !x || !y) return DD_ERR_INVALID_ARG;
    spmv(h->h.lv[0]->A(), x, y, 1, s);
    return DD_OK;
    DD_GUARD_END
}

int dd_info(dd_handle h, dd_info_t* out) {
    DD_GUARD_BEGIN
    if (!h || !out) return DD_ERR_INVALID_ARG;
    Handle& H = h->h;
    if (H.info.k_c == 0 && !H.lv.empty() && H.lv[0]->N > 0) H.info.k_c = coloring_kc(*H.lv[0]);
    *out = H.info;
    return DD_OK;
    DD_GUARD_END
}

void dd_destroy(dd_handle h) { delete h; }


int dd_subdomain_count(dd_handle h, int32_t level, int32_t* N) {
    Level* L = level_of(h, level);
    if (!L || !N) return DD_ERR_INVALID_ARG;
    *N = L->N;
    return DD_OK;
}

int dd_subdomain_sizes(dd_handle h, int32_t level, int32_t* sizes) {
    Level* L = level_of(h, level);
    if (!L || !sizes) return DD_ERR_INVALID_ARG;
    for (int i = 0; i < L->N; ++i) {
        sizes[5 * i] = L->nI[i];
        sizes[5 * i + 1] = L->nG[i];
        sizes[5 * i + 2] = L->nD[i];
        sizes[5 * i + 3] = L->p[i];
        sizes[5 * i + 4] = 0;
    }
    return DD_OK;
}

int dd_subdomain_sets(dd_handle h, int32_t level, int32_t i, int32_t* I, int32_t* Gm, int32_t* Dl) {
    DD_GUARD_BEGIN
    Level* L = level_of(h, level);
    if (!L || i < 0 || i >= L->N) return DD_ERR_INVALID_ARG;
    const int32_t* e = L->ext.p + L->hoffE[i];
    if (I) DD_HIP(hipMemcpy(I, e, L->nI[i] * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (Gm) DD_HIP(hipMemcpy(Gm, e + L->nI[i], L->nG[i] * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (Dl) DD_HIP(hipMemcpy(Dl, e + L->ni[i], L->nD[i] * sizeof(int32_t), hipMemcpyDeviceToHost));
    return DD_OK;
    DD_GUARD_END
}

int dd_subdomain_eigs(dd_handle h, int32_t level, int32_t i, double* mu) {
    Level* L = level_of(h, level);
    if (!L || i < 0 || i >= L->N || !mu) return DD_ERR_INVALID_ARG;
    std::memcpy(mu, L->mu[i].data(), L->mu[i].size() * sizeof(double));
    return DD_OK;
}

int dd_subdomain_basis(dd_handle h, int32_t level, int32_t i, double* Z) {
    DD_GUARD_BEGIN
    Level* L = level_of(h, level);
    if (!L || i < 0 || i >= L->N || !Z) return DD_ERR_INVALID_ARG;
    DD_HIP(hipMemcpy(Z, L->Z.ptr[i], (size_t)L->nI[i] * L->p[i] * sizeof(double), hipMemcpyDeviceToHost));
    return DD_OK;
    DD_GUARD_END
}

int dd_subdomain_sigma1(dd_handle h, int32_t level, double* sigma1) {
    Level* L = level_of(h, level);
    if (!L || !sigma1) return DD_ERR_INVALID_ARG;
    std::memcpy(sigma1, L->sigma1.data(), L->N * sizeof(double));
    return DD_OK;
}

int dd_coarse_matrix(dd_handle h, int32_t level, double* E, int64_t max_n) {
    Level* L = level_of(h, level);
    if (!L || !E) return DD_ERR_INVALID_ARG;
    if (L->nC > max_n || (int64_t)L->Ecopy.size() != L->nC * L->nC) return DD_ERR_INVALID_ARG;
    std::memcpy(E, L->Ecopy.data(), L->Ecopy.size() * sizeof(double));
    return DD_OK;
}

}  // extern "C"
