// Block-sparse supernodal Cholesky of the coarse operator and its solves.
//
// Symbolic phase (host, from sizes and the block graph only): weighted
// minimum-degree ordering of the subdomain blocks and the elimination
// structure struct(k) of every block; blocks along a chain of the
// elimination tree whose structures nest (struct(k) = {next} U struct(next))
// are grouped into supernodes of at most kSnMax columns, so that a dense
// clique (the top of the tree) becomes a few wide panels instead of a long
// sequence of narrow ones.  Numeric phase (device): per tree level, a
// deterministic left-looking update of every panel from its descendants,
// then a batched tall Cholesky of the level's panels; explicit inverses of
// the diagonal blocks turn the triangular solves into matrix-vector products.
// The solves run on the coarse vector permuted to elimination order, where
// every supernode is a contiguous range.
#include "bchol.hpp"

#include <algorithm>
#include <cstdlib>
#include <map>
#include <set>

namespace dd {

constexpr int kSolCh = 256;   // forward: source columns per partial sum
constexpr int kSolRow = 512;  // backward: panel rows per partial sum
constexpr int kSnMax = 4096;  // widest supernode

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
    bstruct.assign(N, {});
    std::vector<char> gone(N, 0);
    const int na = (int)active.size();
    for (int step = 0; step < na; ++step) {
        int best = -1;
        int64_t bw = INT64_MAX;
        for (int i : active) {
            if (gone[i]) continue;
            int64_t wgt = 0;
            for (int j : g[i]) wgt += p[j];
            if (wgt < bw) { bw = wgt; best = i; }
        }
        const int k = best;
        gone[k] = 1;
        pos[k] = step;
        order.push_back(k);
        std::vector<int> S(g[k].begin(), g[k].end());
        bstruct[k] = S;
        for (int a : S) {
            g[a].erase(k);
            for (int b : S)
                if (b != a) g[a].insert(b);
        }
        g[k].clear();
    }
    for (int k : order) std::sort(bstruct[k].begin(), bstruct[k].end(), [&](int a, int b) { return pos[a] < pos[b]; });
    // supernodes (fundamental, width-capped)
    sn.assign(N, -1);
    cof.assign(N, 0);
    members.clear();
    w.clear();
    for (size_t idx = 0; idx < order.size(); ++idx) {
        const int b = order[idx];
        bool merged = false;
        if (idx > 0) {
            const int prev = order[idx - 1];
            const int K = sn[prev];
            const auto& Sp = bstruct[prev];
            const auto& Sb = bstruct[b];
            if (!Sp.empty() && Sp[0] == b && w[K] + p[b] <= kSnMax && Sp.size() == Sb.size() + 1 &&
                std::equal(Sb.begin(), Sb.end(), Sp.begin() + 1)) {
                sn[b] = K;
                cof[b] = w[K];
                w[K] += p[b];
                members[K].push_back(b);
                merged = true;
            }
        }
        if (!merged) {
            sn[b] = (int)members.size();
            cof[b] = 0;
            members.push_back({b});
            w.push_back(p[b]);
        }
    }
    NS = (int)members.size();
    srows.assign(NS, {});
    srowoff.assign(NS, {});
    h.assign(NS, 0);
    start.assign(NS + 1, 0);
    bstart.assign(N, 0);
    for (int K = 0; K < NS; ++K) {
        srows[K] = bstruct[members[K].back()];
        int off = w[K];
        for (int j : srows[K]) {
            srowoff[K].push_back(off);
            off += p[j];
        }
        h[K] = off;
        start[K + 1] = start[K] + w[K];
        for (int b : members[K]) bstart[b] = start[K] + cof[b];
    }
    // elimination-tree levels of the supernodes (children precede parents)
    lev.assign(NS, 0);
    int maxlev = 0;
    for (int K = 0; K < NS; ++K) {
        if (!srows[K].empty()) {
            const int par = sn[srows[K][0]];
            lev[par] = std::max(lev[par], lev[K] + 1);
        }
        maxlev = std::max(maxlev, lev[K]);
    }
    by_level.assign(NS ? maxlev + 1 : 0, {});
    for (int K = 0; K < NS; ++K) by_level[lev[K]].push_back(K);
    poff.assign(NS + 1, 0);
    loff.assign(NS + 1, 0);
    goff.assign(NS + 1, 0);
    flops = 0.0;
    for (int K = 0; K < NS; ++K) {
        poff[K + 1] = poff[K] + (int64_t)h[K] * w[K];
        loff[K + 1] = loff[K] + (int64_t)w[K] * w[K];
        goff[K + 1] = goff[K] + (h[K] - w[K]);
        const double wk = w[K], r = h[K] - w[K];
        flops += wk * wk * wk / 3.0 + r * wk * wk + r * r * wk;
    }
    if (std::getenv("DD_VERBOSE")) {
        fprintf(stderr, "dd: coarse block Cholesky: %d blocks in %d supernodes, n_C %lld, %zu tree levels, panel "
                "entries %lld, flops %.3e\n", na, NS, (long long)nC, by_level.size(), (long long)poff[NS], flops);
        fprintf(stderr, "dd: supernodes per level:");
        for (auto& Lv : by_level) fprintf(stderr, " %zu", Lv.size());
        fprintf(stderr, "\n");
    }
}

double* BlockChol::block(int i, int j, int* ld) const {
    if (p[i] <= 0 || p[j] <= 0 || pos[i] < pos[j]) return nullptr;
    const int K = sn[j];
    int r = -1;
    if (sn[i] == K) {
        r = cof[i];
    } else {
        const auto& S = srows[K];
        for (size_t q = 0; q < S.size(); ++q)
            if (S[q] == i) { r = srowoff[K][q]; break; }
        if (r < 0) return nullptr;
    }
    *ld = h[K];
    return panels.p + poff[K] + r + (int64_t)cof[j] * h[K];
}

void BlockChol::allocate(hipStream_t s) {
    panels.alloc(std::max<int64_t>(1, poff[NS]));
    linv.alloc(std::max<int64_t>(1, loff[NS]));
    fill(panels.p, panels.n, 0.0, s);
    tbuf.alloc(std::max<int64_t>(1, nC));
    ybuf.alloc(std::max<int64_t>(1, nC));
    {
        std::vector<int64_t> hp(std::max<int64_t>(1, nC), 0);
        for (int b = 0; b < N; ++b)
            for (int r = 0; r < p[b]; ++r) hp[yoff[b] + r] = bstart[b] + r;
        perm = upload(hp, s);
    }
    {
        std::vector<int64_t> g(std::max<int64_t>(1, goff[NS]));
        for (int K = 0; K < NS; ++K) {
            int64_t q = goff[K];
            for (int j : srows[K])
                for (int r = 0; r < p[j]; ++r) g[q++] = bstart[j] + r;
        }
        gidx = upload(g, s);
    }
    const int L = (int)by_level.size();
    // factorization update jobs: target (row block b, column block a), a in a
    // supernode K; sources = the descendant supernodes D with a, b in struct(D)
    {
        std::map<std::pair<int, int>, std::vector<std::pair<int, std::pair<int, int>>>> jobs;
        for (int D = 0; D < NS; ++D) {
            const auto& S = srows[D];
            for (size_t ia = 0; ia < S.size(); ++ia)
                for (size_t ib = ia; ib < S.size(); ++ib) jobs[{S[ia], S[ib]}].push_back({D, {(int)ia, (int)ib}});
        }
        upd.clear();
        upd.resize(L);
        upd_src.clear();
        upd_src.resize(L);
        std::vector<std::vector<UpdSrc>> us(L);
        for (auto& kv : jobs) {
            const int a = kv.first.first, b = kv.first.second;
            int ld = 0;
            double* out = block(b, a, &ld);
            if (!out) throw Error(DD_ERR_INTERNAL, "coarse factor: update target outside the structure");
            const int l = lev[sn[a]];
            upd[l].h.push_back(UpdJob{out, ld, p[b], p[a], (int)us[l].size(), (int)kv.second.size(), a == b ? 1 : 0});
            for (auto& src : kv.second) {
                const int D = src.first;
                us[l].push_back(UpdSrc{panels.p + poff[D] + srowoff[D][src.second.second],
                                       panels.p + poff[D] + srowoff[D][src.second.first], h[D], w[D]});
            }
        }
        if (std::getenv("DD_VERBOSE")) {
            for (int l = 0; l < L; ++l) {
                double fl = 0.0, ksum = 0.0;
                int64_t tiles = 0;
                for (auto& j : upd[l].h) {
                    const int64_t tm = ceil_div(j.M, 64), tn = ceil_div(j.N, 64);
                    tiles += j.lower ? tm * (tm + 1) / 2 : tm * tn;
                    for (int q = 0; q < j.nsrc; ++q) {
                        const double K = us[l][j.src0 + q].K;
                        ksum += K;
                        fl += 2.0 * j.M * j.N * K * (j.lower ? 0.5 : 1.0);
                    }
                }
                if (!upd[l].h.empty())
                    fprintf(stderr, "dd: coarse update level %d: %zu jobs, %zu sources (mean K %.0f), %lld tiles, %.3e flops\n",
                            l, upd[l].h.size(), us[l].size(), ksum / std::max<size_t>(1, us[l].size()), (long long)tiles, fl);
            }
        }
        for (int l = 0; l < L; ++l) {
            if (!upd[l].h.empty()) upd[l].sync(s);
            upd_src[l].alloc(std::max<size_t>(1, us[l].size()));
            h2d(upd_src[l].p, us[l].data(), us[l].size(), s);
        }
        DD_HIP(hipStreamSynchronize(s));  // the host source arrays go out of scope
    }
    // forward sources: for supernode K, the descendants D whose struct meets K
    // (a contiguous run of struct(D), since K's blocks are consecutive in pos)
    std::vector<std::vector<std::pair<int, std::pair<int, int>>>> fsrc(NS);  // K -> (D, (q0, q1))
    for (int D = 0; D < NS; ++D) {
        const auto& S = srows[D];
        size_t q = 0;
        while (q < S.size()) {
            const int K = sn[S[q]];
            size_t q1 = q;
            while (q1 + 1 < S.size() && sn[S[q1 + 1]] == K) ++q1;
            fsrc[K].push_back({D, {(int)q, (int)q1}});
            q = q1 + 1;
        }
    }
    sol.clear();
    sol.resize(L);
    sol_src.clear();
    sol_src.resize(L);
    sol_ch.clear();
    sol_ch.resize(L);
    sol_trf.clear();
    sol_trf.resize(L);
    sol_trb.clear();
    sol_trb.resize(L);
    fwd_tiles.assign(L, 0);
    bwd_tiles.assign(L, 0);
    part_len.assign(L, 0);
    std::vector<int32_t> hr;                       // row maps of all forward sources
    std::vector<std::vector<SolSrc>> ss(L);
    std::vector<std::vector<int64_t>> ssroff(L);   // offset of each source's row map in hr
    int64_t pmax = 1, tpmax = 1;
    for (int l = 0; l < L; ++l) {
        int64_t part = 0, tpart = 0;
        for (int K : by_level[l]) {
            const int node = (int)sol[l].h.size();
            SolNode nd{panels.p + poff[K], h[K], w[K], start[K], nullptr, (int)sol_ch[l].h.size(), 0,
                       ceil_div(h[K] - w[K], kSolRow), part};
            for (auto& fs : fsrc[K]) {
                const int D = fs.first, q0 = fs.second.first, q1 = fs.second.second;
                const int64_t roff = (int64_t)hr.size();
                int rows = 0;
                for (int q = q0; q <= q1; ++q) {
                    const int b = srows[D][q];
                    for (int r = 0; r < p[b]; ++r) hr.push_back(cof[b] + r);
                    rows += p[b];
                }
                const int lsrc = (int)ss[l].size();
                ss[l].push_back(SolSrc{panels.p + poff[D] + srowoff[D][q0], h[D], w[D], rows, start[D], nullptr});
                ssroff[l].push_back(roff);
                for (int c0 = 0; c0 < w[D]; c0 += kSolCh) {
                    sol_ch[l].h.push_back(SolChunk{node, lsrc, c0, std::min(w[D], c0 + kSolCh)});
                    fwd_tiles[l] += ceil_div(rows, 64);
                }
            }
            nd.nfch = (int)sol_ch[l].h.size() - nd.fch0;
            nd.gidx = gidx.p + goff[K];
            part += (int64_t)w[K] * std::max(nd.nfch, nd.nbch);
            bwd_tiles[l] += (int64_t)nd.nbch * ceil_div(w[K], 64);
            sol[l].h.push_back(nd);
            tpart += trmv_part_size(w[K]);
        }
        part_len[l] = part;
        pmax = std::max(pmax, part);
        tpmax = std::max(tpmax, tpart);
    }
    if (hr.empty()) hr.push_back(0);
    ridx = upload(hr, s);
    pbuf.alloc(pmax);
    trpart.alloc(tpmax);
    for (int l = 0; l < L; ++l) {
        for (size_t q = 0; q < ss[l].size(); ++q) ss[l][q].ridx = ridx.p + ssroff[l][q];
        int64_t tp = 0;
        for (int K : by_level[l]) {
            // forward: y_K = L_KK^{-1} t_K;  backward: y_K = L_KK^{-T} t_K
            sol_trf[l].h.push_back(TrmvItem{linv.p + loff[K], w[K], w[K], tbuf.p + start[K], ybuf.p + start[K], trpart.p + tp});
            sol_trb[l].h.push_back(TrmvItem{linv.p + loff[K], w[K], w[K], ybuf.p + start[K], tbuf.p + start[K], trpart.p + tp});
            tp += trmv_part_size(w[K]);
        }
        sol[l].sync(s);
        sol_trf[l].sync(s);
        sol_trb[l].sync(s);
        sol_src[l].alloc(std::max<size_t>(1, ss[l].size()));
        h2d(sol_src[l].p, ss[l].data(), ss[l].size(), s);
        if (sol_ch[l].h.empty()) sol_ch[l].h.push_back(SolChunk{0, 0, 0, 0});
        sol_ch[l].sync(s);
    }
    DD_HIP(hipStreamSynchronize(s));
}

// out -= sum_src A_src B_src^T over 64x64 output tiles
struct OpBUpd {
    const UpdJob* jobs;
    const UpdSrc* src;
    __device__ int tiles(int b) const {
        const int tm = (jobs[b].M + 63) / 64, tn = (jobs[b].N + 63) / 64;
        return jobs[b].lower ? tm * (tm + 1) / 2 : tm * tn;
    }
    __device__ void operator()(int b, int t) const {
        __shared__ TileSmemC sm;
        const UpdJob J = jobs[b];
        const int tm = (J.M + 63) / 64;
        int i0, j0;
        if (J.lower) {  // tile (ti, tj), ti >= tj, column by column
            int tj = 0, r = t;
            while (r >= tm - tj) {
                r -= tm - tj;
                ++tj;
            }
            i0 = (tj + r) * 64;
            j0 = tj * 64;
        } else {
            i0 = (t % tm) * 64;
            j0 = (t / tm) * 64;
        }
        double4_t acc[2][2];
        acc_zero(acc);
        for (int q = 0; q < J.nsrc; ++q) {
            const UpdSrc S = src[J.src0 + q];
            mfma_tile_64<false, true>(S.A, S.ld, S.B, S.ld, J.M, J.N, S.K, i0, j0, sm.t, acc);
        }
        acc_store_coalesced(acc, sm, [&](int r, int c, double v) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < J.M && gj < J.N) J.out[gi + (int64_t)gj * J.ldo] -= v;
        });
    }
};

int BlockChol::factor(hipStream_t s) {
    const int L = (int)by_level.size();
    for (int l = 0; l < L; ++l) {
        if (!upd[l].h.empty()) {
            int64_t tot = 0;
            for (auto& j : upd[l].h) {
                const int64_t tm = ceil_div(j.M, 64), tn = ceil_div(j.N, 64);
                tot += j.lower ? tm * (tm + 1) / 2 : tm * tn;
            }
            launch_tiles(OpBUpd{upd[l].d.p, upd_src[l].p}, upd[l].size(), tot, s, "bchol_update");
        }
        Batch<DMat> pn, dg, iv;
        for (int K : by_level[l]) {
            pn.h.push_back(DMat{panels.p + poff[K], h[K], h[K], w[K]});
            dg.h.push_back(DMat{panels.p + poff[K], h[K], w[K], w[K]});
            iv.h.push_back(DMat{linv.p + loff[K], w[K], w[K], w[K]});
        }
        pn.sync(s);
        dg.sync(s);
        iv.sync(s);
        DBuf<int32_t> li(pn.size());
        DD_HIP(hipMemsetAsync(li.p, 0, pn.size() * sizeof(int32_t), s));
        potrf_vb(pn, li.p, s);
        set_identity_vb(iv, 1.0, s);
        trsm_vb(dg, iv, false, s, true);  // L_KK^{-1}
        std::vector<int32_t> hl(pn.size());
        DD_HIP(hipMemcpyAsync(hl.data(), li.p, pn.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DD_HIP(hipStreamSynchronize(s));
        for (size_t q = 0; q < hl.size(); ++q)
            if (hl[q]) return members[by_level[l][q]][0] + 1;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// solves (on the permuted coarse vector ybuf)
// ---------------------------------------------------------------------------
__global__ void k_perm_gather(const double* y, const int64_t* perm, int64_t n, double* yp) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        yp[perm[q]] = y[q];
}
__global__ void k_perm_scatter(const double* yp, const int64_t* perm, int64_t n, double* y) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        y[q] = yp[perm[q]];
}

// forward, pass 1: partial sums of L_{K,D} x_D over one column chunk of one
// descendant D (its rows that fall in K), 64 rows per workgroup, written to
// the rows of K they belong to (the other rows of the chunk's slice stay 0).
struct OpFwdPart {
    const SolNode* nodes;
    const SolSrc* src;
    const SolChunk* ch;
    const double* x;
    double* part;
    __device__ int tiles(int g) const { return (ch[g].c1 > ch[g].c0) ? (src[ch[g].src].rows + 63) / 64 : 0; }
    __device__ void operator()(int g, int tile) const {
        __shared__ double red[4][64];
        const SolChunk C = ch[g];
        const SolNode nd = nodes[C.node];
        const SolSrc S = src[C.src];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int r = tile * 64 + lane;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;  // four loads in flight per lane
        if (r < S.rows) {
            const double* Lr = S.L + r;
            const double* xs = x + S.xoff;
            int c = C.c0 + wv;
            for (; c + 12 < C.c1; c += 16) {
                a0 += Lr[(int64_t)c * S.ld] * xs[c];
                a1 += Lr[(int64_t)(c + 4) * S.ld] * xs[c + 4];
                a2 += Lr[(int64_t)(c + 8) * S.ld] * xs[c + 8];
                a3 += Lr[(int64_t)(c + 12) * S.ld] * xs[c + 12];
            }
            for (; c < C.c1; c += 4) a0 += Lr[(int64_t)c * S.ld] * xs[c];
        }
        red[wv][lane] = (a0 + a1) + (a2 + a3);
        __syncthreads();
        if (wv == 0 && r < S.rows)
            part[nd.part0 + (int64_t)(g - nd.fch0) * nd.w + S.ridx[r]] =
                (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    }
};
// pass 2 (both directions): t_K = y_K - sum of the node's partials.  A tile
// is 64 rows (lane = row); wave wv sums the partials q = wv, wv + 4, ... with
// two accumulators, and the four wave sums are added in a fixed order.
struct OpSolRed {
    const SolNode* nodes;
    const double* part;
    const double* y;
    double* t;
    int backward;
    __device__ int tiles(int b) const { return (nodes[b].w + 63) / 64; }
    __device__ void operator()(int b, int tile) const {
        __shared__ double red[4][64];
        const SolNode nd = nodes[b];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int r = tile * 64 + lane;
        const int nch = backward ? nd.nbch : nd.nfch;
        double a0 = 0.0, a1 = 0.0;
        if (r < nd.w) {
            const double* p = part + nd.part0 + r;
            int q = wv;
            for (; q + 4 < nch; q += 8) {
                a0 += p[(int64_t)q * nd.w];
                a1 += p[(int64_t)(q + 4) * nd.w];
            }
            for (; q < nch; q += 4) a0 += p[(int64_t)q * nd.w];
        }
        red[wv][lane] = a0 + a1;
        __syncthreads();
        if (wv == 0 && r < nd.w)
            t[nd.start + r] = y[nd.start + r] - ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]));
    }
};
// backward, pass 1: partial column dots of panel K over one chunk of rows below the diagonal block
struct OpBwdPart {
    const SolNode* nodes;
    const double* x;
    double* part;
    __device__ int tiles(int b) const { return nodes[b].nbch * ((nodes[b].w + 63) / 64); }
    __device__ void operator()(int b, int tile) const {
        __shared__ double xs[kSolRow];  // x at the chunk's rows, gathered once
        const SolNode nd = nodes[b];
        const int nct = (nd.w + 63) / 64;
        const int rc = tile / nct, ct = tile % nct;
        const int q0 = nd.w + rc * kSolRow, q1 = min(nd.h, q0 + kSolRow);
        for (int q = q0 + (int)threadIdx.x; q < q1; q += blockDim.x) xs[q - q0] = x[nd.gidx[q - nd.w]];
        __syncthreads();
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        // wave wv: columns ct*64 + 16 wv + k, k < 16, all sixteen in flight together
        const int c0 = ct * 64 + 16 * wv;
        const int nk = min(16, nd.w - c0);
        if (nk <= 0) return;
        const double* col = nd.panel + (int64_t)c0 * nd.h;
        double acc[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0;
        for (int q = q0 + lane; q < q1; q += 64) {
            const double xv = xs[q - q0];
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < nk) acc[k] += col[q + (int64_t)k * nd.h] * xv;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double v = wave_sum(acc[k]);
            if (lane == 0 && k < nk) part[nd.part0 + (int64_t)rc * nd.w + c0 + k] = v;
        }
    }
};

void BlockChol::solve(double* y, hipStream_t s) {
    if (nC <= 0) return;
    const int grid = (int)std::min<int64_t>((nC + 255) / 256, 4096);
    hipLaunchKernelGGL(k_perm_gather, dim3(grid), dim3(256), 0, s, y, perm.p, nC, ybuf.p);
    launch_check("bchol_perm");
    const int L = (int)by_level.size();
    for (int l = 0; l < L; ++l) {
        int64_t tot4 = 0;
        for (auto& nd : sol[l].h) tot4 += ceil_div(nd.w, 64);
        if (fwd_tiles[l] > 0) {
            fill(pbuf.p, part_len[l], 0.0, s);
            launch_tiles(OpFwdPart{sol[l].d.p, sol_src[l].p, sol_ch[l].d.p, ybuf.p, pbuf.p}, sol_ch[l].size(),
                         fwd_tiles[l], s, "bchol_fwd_part");
        }
        launch_tiles(OpSolRed{sol[l].d.p, pbuf.p, ybuf.p, tbuf.p, 0}, sol[l].size(), tot4, s, "bchol_fwd_red");
        trmv_n_vb(sol_trf[l], s);  // y_K = L_KK^{-1} t_K
    }
    for (int l = L - 1; l >= 0; --l) {
        int64_t tot4 = 0;
        for (auto& nd : sol[l].h) tot4 += ceil_div(nd.w, 64);
        if (bwd_tiles[l] > 0)
            launch_tiles(OpBwdPart{sol[l].d.p, ybuf.p, pbuf.p}, sol[l].size(), bwd_tiles[l], s, "bchol_bwd_part");
        launch_tiles(OpSolRed{sol[l].d.p, pbuf.p, ybuf.p, tbuf.p, 1}, sol[l].size(), tot4, s, "bchol_bwd_red");
        trmv_t_vb(sol_trb[l], s);  // y_K = L_KK^{-T} t_K
    }
    hipLaunchKernelGGL(k_perm_scatter, dim3(grid), dim3(256), 0, s, ybuf.p, perm.p, nC, y);
    launch_check("bchol_perm");
}

}  // namespace dd
