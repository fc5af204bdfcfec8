// Block-sparse (supernodal) Cholesky of the coarse operator and its solves.
//
// Symbolic phase (host, from sizes and the block graph only): weighted
// minimum-degree ordering of the subdomain blocks, elimination structure
// struct(k) (the blocks below the diagonal in block column k of L), the
// elimination-tree levels, and the panel layout.  Numeric phase (device):
// per level, a deterministic left-looking block update of every panel of the
// level followed by a batched tall Cholesky of those panels; explicit
// inverses of the diagonal blocks serve the triangular solves.
#include "bchol.hpp"

#include <algorithm>
#include <cstdlib>
#include <set>

namespace dd {

constexpr int kSolCh = 256;   // forward: columns per partial sum
constexpr int kSolRow = 512;  // backward: panel rows per partial sum

void BlockChol::symbolic(const std::vector<uint8_t>& adj, const std::vector<int>& p_,
                         const std::vector<int64_t>& yoff_) {
    N = (int)p_.size();
    p = p_;
    yoff = yoff_;
    nC = yoff.back();
    std::vector<std::set<int>> g(N);
    std::vector<int> active;
    for (int i = 0; i < N; ++i) {
        if (p[i] <= 0) continue;
        active.push_back(i);
        for (int j = 0; j < N; ++j)
            if (j != i && p[j] > 0 && adj[(size_t)i * N + j]) g[i].insert(j);
    }
    // weighted minimum (external) degree, ties -> lowest id
    pos.assign(N, -1);
    order.clear();
    strct.assign(N, {});
    std::vector<char> gone(N, 0);
    const int na = (int)active.size();
    for (int step = 0; step < na; ++step) {
        int best = -1;
        int64_t bw = INT64_MAX;
        for (int i : active) {
            if (gone[i]) continue;
            int64_t w = 0;
            for (int j : g[i]) w += p[j];
            if (w < bw) { bw = w; best = i; }
        }
        const int k = best;
        gone[k] = 1;
        pos[k] = step;
        order.push_back(k);
        std::vector<int> S(g[k].begin(), g[k].end());
        strct[k] = S;
        for (int a : S) {
            g[a].erase(k);
            for (int b : S)
                if (b != a) g[a].insert(b);
        }
        g[k].clear();
    }
    // sort struct by elimination position; row offsets; heights
    rowoff.assign(N, {});
    h.assign(N, 0);
    for (int k : order) {
        std::sort(strct[k].begin(), strct[k].end(), [&](int a, int b) { return pos[a] < pos[b]; });
        int off = p[k];
        rowoff[k].resize(strct[k].size());
        for (size_t q = 0; q < strct[k].size(); ++q) {
            rowoff[k][q] = off;
            off += p[strct[k][q]];
        }
        h[k] = off;
    }
    // elimination tree levels: parent = first block of struct(k)
    lev.assign(N, 0);
    int maxlev = 0;
    for (int k : order) {
        if (!strct[k].empty()) {
            const int par = strct[k][0];
            lev[par] = std::max(lev[par], lev[k] + 1);
        }
        maxlev = std::max(maxlev, lev[k]);
    }
    by_level.assign(na ? maxlev + 1 : 0, {});
    for (int k : order) by_level[lev[k]].push_back(k);
    // offsets
    poff.assign(N + 1, 0);
    loff.assign(N + 1, 0);
    goff.assign(N + 1, 0);
    int64_t P = 0, Lo = 0, G = 0;
    flops = 0.0;
    for (int i = 0; i < N; ++i) {
        poff[i] = P;
        loff[i] = Lo;
        goff[i] = G;
        if (p[i] > 0) {
            P += (int64_t)h[i] * p[i];
            Lo += (int64_t)p[i] * p[i];
            G += h[i] - p[i];
            const double pk = p[i], hk = h[i];
            flops += pk * pk * pk / 3.0 + (hk - pk) * pk * pk + (hk - pk) * (hk - pk) * pk;
        }
    }
    poff[N] = P;
    loff[N] = Lo;
    goff[N] = G;
    if (std::getenv("DD_VERBOSE")) {
        fprintf(stderr, "dd: coarse block Cholesky: %d blocks, n_C %lld, %zu tree levels, panel entries %lld, "
                "flops %.3e\n", na, (long long)nC, by_level.size(), (long long)P, flops);
        fprintf(stderr, "dd: nodes per level:");
        for (auto& L : by_level) fprintf(stderr, " %zu", L.size());
        fprintf(stderr, "\n");
    }
}

static int row_offset(const BlockChol& B, int k, int j) {
    if (j == k) return 0;
    const auto& S = B.strct[k];
    for (size_t q = 0; q < S.size(); ++q)
        if (S[q] == j) return B.rowoff[k][q];
    return -1;
}

double* BlockChol::block(int i, int j, int* ld) const {
    const int r = row_offset(*this, j, i);
    if (r < 0) return nullptr;
    *ld = h[j];
    return panels.p + poff[j] + r;
}

void BlockChol::allocate(hipStream_t s) {
    panels.alloc(std::max<int64_t>(1, poff[N]));
    linv.alloc(std::max<int64_t>(1, loff[N]));
    fill(panels.p, panels.n, 0.0, s);
    tbuf.alloc(std::max<int64_t>(1, nC));
    // backward gather indices: panel row q >= p_k of node k -> coarse index
    std::vector<int64_t> g(std::max<int64_t>(1, goff[N]));
    for (int k = 0; k < N; ++k) {
        if (p[k] <= 0) continue;
        int64_t q = goff[k];
        for (int j : strct[k])
            for (int r = 0; r < p[j]; ++r) g[q++] = yoff[j] + r;
    }
    gidx.alloc(g.size());
    h2d(gidx.p, g.data(), g.size(), s);
    // factorization update jobs: for node k and block row j in {k} U struct(k),
    // sources are the descendants d with k, j in struct(d)
    const int L = (int)by_level.size();
    std::vector<std::vector<std::vector<int>>> srcs(N);  // srcs[k][q]: q = 0 diag, q >= 1 struct index
    for (int k = 0; k < N; ++k)
        if (p[k] > 0) srcs[k].assign(strct[k].size() + 1, {});
    for (int d : order) {
        const auto& S = strct[d];
        for (size_t a = 0; a < S.size(); ++a) {
            const int k = S[a];
            srcs[k][0].push_back(d);
            for (size_t b = a + 1; b < S.size(); ++b) {
                const int j = S[b];
                // j in struct(k) (elimination-tree property); find its index
                const auto& Sk = strct[k];
                const int q = (int)(std::find(Sk.begin(), Sk.end(), j) - Sk.begin());
                srcs[k][q + 1].push_back(d);
            }
        }
    }
    upd.clear();
    upd.resize(L);
    upd_src.clear();
    upd_src.resize(L);
    sol.clear();
    sol.resize(L);
    sol_src.clear();
    sol_src.resize(L);
    sol_ch.clear();
    sol_ch.resize(L);
    fwd_tiles.assign(L, 0);
    bwd_tiles.assign(L, 0);
    int64_t pmax = 1;
    for (int l = 0; l < L; ++l) {
        std::vector<UpdSrc> us;
        std::vector<SolSrc> ss;
        int64_t part = 0;
        for (int k : by_level[l]) {
            const int nq = (int)strct[k].size() + 1;
            for (int q = 0; q < nq; ++q) {
                const int j = (q == 0) ? k : strct[k][q - 1];
                const auto& D = srcs[k][q];
                if (D.empty()) continue;
                UpdJob job{panels.p + poff[k] + (q == 0 ? 0 : rowoff[k][q - 1]), h[k], p[j], p[k], (int)us.size(),
                           (int)D.size()};
                for (int d : D) {
                    const int rj = row_offset(*this, d, j), rk = row_offset(*this, d, k);
                    us.push_back(UpdSrc{panels.p + poff[d] + rj, panels.p + poff[d] + rk, h[d], p[d]});
                }
                upd[l].h.push_back(job);
            }
            const int node = (int)sol[l].h.size();
            SolNode sn{panels.p + poff[k], h[k], p[k], linv.p + loff[k], yoff[k], (int)ss.size(),
                       (int)srcs[k][0].size(), gidx.p + goff[k], (int)sol_ch[l].h.size(), 0, 0, part};
            for (int d : srcs[k][0]) {
                const int qi = (int)ss.size();
                ss.push_back(SolSrc{panels.p + poff[d] + row_offset(*this, d, k), h[d], p[d], yoff[d]});
                for (int c0 = 0; c0 < p[d]; c0 += kSolCh) sol_ch[l].h.push_back(SolChunk{node, qi, c0, std::min(p[d], c0 + kSolCh)});
            }
            sn.nfch = (int)sol_ch[l].h.size() - sn.fch0;
            sn.nbch = ceil_div(h[k] - p[k], kSolRow);
            part += (int64_t)p[k] * std::max(sn.nfch, sn.nbch);
            fwd_tiles[l] += (int64_t)sn.nfch * ceil_div(p[k], 64);
            bwd_tiles[l] += (int64_t)sn.nbch * ceil_div(p[k], 64);
            sol[l].h.push_back(sn);
        }
        pmax = std::max(pmax, part);
        if (!upd[l].h.empty()) upd[l].sync(s);
        upd_src[l].alloc(std::max<size_t>(1, us.size()));
        h2d(upd_src[l].p, us.data(), us.size(), s);
        sol[l].sync(s);
        sol_src[l].alloc(std::max<size_t>(1, ss.size()));
        h2d(sol_src[l].p, ss.data(), ss.size(), s);
        if (sol_ch[l].h.empty()) sol_ch[l].h.push_back(SolChunk{0, 0, 0, 0});
        sol_ch[l].sync(s);
    }
    pbuf.alloc(pmax);
    DD_HIP(hipStreamSynchronize(s));
}

// out -= sum_src A_src B_src^T over 64x64 output tiles
struct OpBUpd {
    const UpdJob* jobs;
    const UpdSrc* src;
    __device__ int tiles(int b) const { return ((jobs[b].M + 63) / 64) * ((jobs[b].N + 63) / 64); }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmem sm;
        const UpdJob J = jobs[b];
        const int tm = (J.M + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        double4_t acc[2][2];
        acc_zero(acc);
        for (int q = 0; q < J.nsrc; ++q) {
            const UpdSrc S = src[J.src0 + q];
            mfma_tile_64<false, true>(S.A, S.ld, S.B, S.ld, J.M, J.N, S.K, i0, j0, sm, acc);
        }
        acc_foreach(acc, [&](int r, int c, double v) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < J.M && gj < J.N) J.out[gi + (int64_t)gj * J.ldo] -= v;
        });
    }
};

int BlockChol::factor(hipStream_t s) {
    DBuf<int32_t> info(std::max(1, N));
    DD_HIP(hipMemsetAsync(info.p, 0, std::max(1, N) * sizeof(int32_t), s));
    const int L = (int)by_level.size();
    for (int l = 0; l < L; ++l) {
        if (!upd[l].h.empty()) {
            int64_t tot = 0;
            for (auto& j : upd[l].h) tot += (int64_t)ceil_div(j.M, 64) * ceil_div(j.N, 64);
            launch_tiles(OpBUpd{upd[l].d.p, upd_src[l].p}, upd[l].size(), tot, s, "bchol_update");
        }
        Batch<DMat> pn, dg, iv;
        for (int k : by_level[l]) {
            pn.h.push_back(DMat{panels.p + poff[k], h[k], h[k], p[k]});
            dg.h.push_back(DMat{panels.p + poff[k], h[k], p[k], p[k]});
            iv.h.push_back(DMat{linv.p + loff[k], p[k], p[k], p[k]});
        }
        pn.sync(s);
        dg.sync(s);
        iv.sync(s);
        // info index: position within the level; remapped below on failure
        DBuf<int32_t> li(pn.size());
        DD_HIP(hipMemsetAsync(li.p, 0, pn.size() * sizeof(int32_t), s));
        potrf_vb(pn, li.p, s);
        set_identity_vb(iv, 1.0, s);
        trsm_vb(dg, iv, false, s);  // L_kk^{-1}
        std::vector<int32_t> hl(pn.size());
        DD_HIP(hipMemcpyAsync(hl.data(), li.p, pn.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DD_HIP(hipStreamSynchronize(s));
        for (size_t q = 0; q < hl.size(); ++q)
            if (hl[q]) return by_level[l][q] + 1;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------
// forward, pass 1: partial sums of L_{k,d} y_d over one column chunk of one
// descendant d (rows of block k inside panel d), 64 rows per workgroup.
struct OpFwdPart {
    const SolNode* nodes;
    const SolSrc* src;
    const SolChunk* ch;
    const double* y;
    double* part;
    __device__ int tiles(int g) const { return (nodes[ch[g].node].p + 63) / 64 * (ch[g].c1 > ch[g].c0); }
    __device__ void operator()(int g, int tile) const {
        __shared__ double red[4][64];
        const SolChunk C = ch[g];
        const SolNode nd = nodes[C.node];
        const SolSrc S = src[C.src];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int r = tile * 64 + lane;
        double acc = 0.0;
        if (r < nd.p)
            for (int c = C.c0 + wv; c < C.c1; c += 4) acc += S.L[r + (int64_t)c * S.ld] * y[S.yoff + c];
        red[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && r < nd.p)
            part[nd.part0 + (int64_t)(g - nd.fch0) * nd.p + r] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    }
};
// forward, pass 2: t_k = y_k - sum of the partials (in chunk order)
struct OpFwdRed {
    const SolNode* nodes;
    const double* part;
    const double* y;
    double* t;
    __device__ int tiles(int b) const { return (nodes[b].p + 255) / 256; }
    __device__ void operator()(int b, int tile) const {
        const SolNode nd = nodes[b];
        const int r = tile * 256 + threadIdx.x;
        if (r >= nd.p) return;
        double acc = 0.0;
        for (int q = 0; q < nd.nfch; ++q) acc += part[nd.part0 + (int64_t)q * nd.p + r];
        t[nd.yoff + r] = y[nd.yoff + r] - acc;
    }
};
// forward, pass 3: y_k = L_kk^{-1} t_k
struct OpFwdY {
    const SolNode* nodes;
    const double* t;
    double* y;
    __device__ int tiles(int b) const { return (nodes[b].p + 63) / 64; }
    __device__ void operator()(int b, int tile) const {
        __shared__ double red[4][64];
        const SolNode nd = nodes[b];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int r = tile * 64 + lane;
        double acc = 0.0;
        if (r < nd.p)
            for (int c = wv; c <= r; c += 4) acc += nd.linv[r + (int64_t)c * nd.p] * t[nd.yoff + c];
        red[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && r < nd.p) y[nd.yoff + r] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    }
};
// backward, pass 1: partial column dots of panel k over one chunk of rows below the diagonal block
struct OpBwdPart {
    const SolNode* nodes;
    const double* x;
    double* part;
    __device__ int tiles(int b) const { return nodes[b].nbch * ((nodes[b].p + 63) / 64); }
    __device__ void operator()(int b, int tile) const {
        const SolNode nd = nodes[b];
        const int nct = (nd.p + 63) / 64;
        const int rc = tile / nct, ct = tile % nct;
        const int q0 = nd.p + rc * kSolRow, q1 = min(nd.h, q0 + kSolRow);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int cc = wv; cc < 64; cc += 4) {
            const int c = ct * 64 + cc;
            if (c >= nd.p) break;
            const double* col = nd.panel + (int64_t)c * nd.h;
            double acc = 0.0;
            for (int q = q0 + lane; q < q1; q += 64) acc += col[q] * x[nd.gidx[q - nd.p]];
            acc = wave_sum(acc);
            if (lane == 0) part[nd.part0 + (int64_t)rc * nd.p + c] = acc;
        }
    }
};
struct OpBwdRed {
    const SolNode* nodes;
    const double* part;
    const double* x;
    double* t;
    __device__ int tiles(int b) const { return (nodes[b].p + 255) / 256; }
    __device__ void operator()(int b, int tile) const {
        const SolNode nd = nodes[b];
        const int c = tile * 256 + threadIdx.x;
        if (c >= nd.p) return;
        double acc = 0.0;
        for (int q = 0; q < nd.nbch; ++q) acc += part[nd.part0 + (int64_t)q * nd.p + c];
        t[nd.yoff + c] = x[nd.yoff + c] - acc;
    }
};
// backward, pass 3: x_k = L_kk^{-T} t_k (column dots of the inverse)
struct OpBwdX {
    const SolNode* nodes;
    const double* t;
    double* x;
    __device__ int tiles(int b) const { return (nodes[b].p + 63) / 64; }
    __device__ void operator()(int b, int tile) const {
        const SolNode nd = nodes[b];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int cc = wv; cc < 64; cc += 4) {
            const int c = tile * 64 + cc;
            if (c >= nd.p) break;
            const double* col = nd.linv + (int64_t)c * nd.p;
            double acc = 0.0;
            for (int r = c + lane; r < nd.p; r += 64) acc += col[r] * t[nd.yoff + r];
            acc = wave_sum(acc);
            if (lane == 0) x[nd.yoff + c] = acc;
        }
    }
};

void BlockChol::solve(double* y, hipStream_t s) {
    const int L = (int)by_level.size();
    for (int l = 0; l < L; ++l) {
        int64_t tot = 0, tot4 = 0;
        for (auto& nd : sol[l].h) {
            tot += ceil_div(nd.p, 64);
            tot4 += ceil_div(nd.p, 256);
        }
        if (fwd_tiles[l] > 0)
            launch_tiles(OpFwdPart{sol[l].d.p, sol_src[l].p, sol_ch[l].d.p, y, pbuf.p}, sol_ch[l].size(), fwd_tiles[l], s,
                         "bchol_fwd_part");
        launch_tiles(OpFwdRed{sol[l].d.p, pbuf.p, y, tbuf.p}, sol[l].size(), tot4, s, "bchol_fwd_red");
        launch_tiles(OpFwdY{sol[l].d.p, tbuf.p, y}, sol[l].size(), tot, s, "bchol_fwd_y");
    }
    for (int l = L - 1; l >= 0; --l) {
        int64_t tot = 0, tot4 = 0;
        for (auto& nd : sol[l].h) {
            tot += ceil_div(nd.p, 64);
            tot4 += ceil_div(nd.p, 256);
        }
        if (bwd_tiles[l] > 0) launch_tiles(OpBwdPart{sol[l].d.p, y, pbuf.p}, sol[l].size(), bwd_tiles[l], s, "bchol_bwd_part");
        launch_tiles(OpBwdRed{sol[l].d.p, pbuf.p, y, tbuf.p}, sol[l].size(), tot4, s, "bchol_bwd_red");
        launch_tiles(OpBwdX{sol[l].d.p, tbuf.p, y}, sol[l].size(), tot, s, "bchol_bwd_x");
    }
}

}  // namespace dd
