// Symbolic analysis of the local factors (host).
//
// Each subgraph's port-augmented matrix K_k of eq. (5.8) has the sparsity of its
// piece A~_k (the ports only touch the diagonal), so the analysis depends on
// the local structure alone and is shared by all subgraphs with the same one.
//
//  * Ordering: nested dissection by coordinate bisection; the separator of a
//    part is the vertex cover of the cut edges on the lower side.  Without
//    coordinates a BFS-level coordinate from a pseudo-peripheral vertex is used.
//  * Supernodes: the column blocks of the dissection tree (separators and
//    leaves), eliminated as dense blocks.  The front of supernode s is
//    cols(s) + R_s, R_s = rows coupled to cols(s) after eliminating everything
//    before it; the assembly parent of s is the supernode holding min(R_s).
//  * Level order: supernodes are renumbered by assembly-tree level (leaves
//    first).  Subtrees at one level are independent, so this is a valid
//    elimination order with the same fill, and every level becomes one
//    contiguous column range that a workgroup processes in parallel.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "vtm_internal.hpp"

namespace vtm {
namespace {

struct LocalGraph {
    int32_t nk;
    std::vector<int32_t> ptr, adj;  // without the diagonal
    std::vector<double> xyz;        // nk x 3 coordinates (zeros if none)
    bool has_coords;
};

void bfs_levels(const LocalGraph &g, const std::vector<int32_t> &verts, std::vector<int32_t> &mark, int32_t tag,
                std::vector<double> &coord) {
    // coord[v] = BFS distance from a pseudo-peripheral vertex inside `verts` (mark[v] == tag)
    std::vector<int32_t> dist(verts.size()), queue;
    std::unordered_map<int32_t, int32_t> loc;
    for (size_t i = 0; i < verts.size(); ++i) loc[verts[i]] = (int32_t)i;
    auto run = [&](int32_t src) {
        std::fill(dist.begin(), dist.end(), -1);
        queue.assign(1, src);
        dist[loc[src]] = 0;
        int32_t last = src;
        for (size_t h = 0; h < queue.size(); ++h) {
            int32_t v = queue[h];
            last = v;
            for (int32_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
                int32_t u = g.adj[e];
                if (mark[u] != tag) continue;
                int32_t &du = dist[loc[u]];
                if (du < 0) { du = dist[loc[v]] + 1; queue.push_back(u); }
            }
        }
        return last;
    };
    int32_t far = run(verts[0]);
    run(far);
    int32_t mx = 0;
    for (int32_t d : dist) mx = std::max(mx, d);
    for (size_t i = 0; i < verts.size(); ++i) coord[verts[i]] = dist[i] < 0 ? mx + 1 : dist[i];
}

// Nested dissection: appends supernode column blocks (local vertex lists) in postorder.
void dissect(const LocalGraph &g, std::vector<int32_t> verts, int leaf, std::vector<int32_t> &mark, int32_t &tag,
             std::vector<double> &coord, std::vector<std::vector<int32_t>> &blocks) {
    if ((int)verts.size() <= leaf) {
        std::sort(verts.begin(), verts.end());
        blocks.push_back(std::move(verts));
        return;
    }
    int ax = 0, naxes = 3;
    const double *X = g.xyz.data();
    std::vector<double> c1;
    if (!g.has_coords) {
        ++tag;
        for (int32_t v : verts) mark[v] = tag;
        bfs_levels(g, verts, mark, tag, coord);
        naxes = 1;
    }
    auto crd = [&](int32_t v, int a) { return g.has_coords ? X[3 * v + a] : coord[v]; };
    double best = -1.0;
    for (int a = 0; a < naxes; ++a) {
        double lo = crd(verts[0], a), hi = lo;
        for (int32_t v : verts) { lo = std::min(lo, crd(v, a)); hi = std::max(hi, crd(v, a)); }
        if (hi - lo > best) { best = hi - lo; ax = a; }
    }
    if (best <= 0.0) {
        std::sort(verts.begin(), verts.end());
        blocks.push_back(std::move(verts));
        return;
    }
    std::sort(verts.begin(), verts.end(), [&](int32_t u, int32_t v) {
        double cu = crd(u, ax), cv = crd(v, ax);
        return cu < cv || (cu == cv && u < v);
    });
    size_t h = verts.size() / 2;
    while (h > 0 && crd(verts[h - 1], ax) == crd(verts[h], ax)) --h;
    if (h == 0) {
        while (h < verts.size() && crd(verts[h], ax) == crd(verts[0], ax)) ++h;
    }
    ++tag;
    const int32_t rtag = tag;
    for (size_t i = h; i < verts.size(); ++i) mark[verts[i]] = rtag;
    std::vector<int32_t> left, sep, right(verts.begin() + h, verts.end());
    for (size_t i = 0; i < h; ++i) {
        int32_t v = verts[i];
        bool cut = false;
        for (int32_t e = g.ptr[v]; e < g.ptr[v + 1] && !cut; ++e) cut = mark[g.adj[e]] == rtag;
        (cut ? sep : left).push_back(v);
    }
    if (!left.empty()) dissect(g, std::move(left), leaf, mark, tag, coord, blocks);
    if (!right.empty()) dissect(g, std::move(right), leaf, mark, tag, coord, blocks);
    if (!sep.empty()) {
        std::sort(sep.begin(), sep.end());
        blocks.push_back(std::move(sep));
    }
}

uint64_t structure_hash(const Partition &P, int32_t k) {
    uint64_t h = 1469598103934665603ULL;
    auto mix = [&](uint64_t x) { h = (h ^ x) * 1099511628211ULL; };
    const int64_t b = P.loc_ptr[k], nk = P.loc_ptr[k + 1] - b;
    mix((uint64_t)nk);
    const int64_t e0 = P.lrp[b];
    for (int64_t i = 0; i <= nk; ++i) mix((uint64_t)(P.lrp[b + i] - e0));
    for (int64_t e = e0; e < P.lrp[b + nk]; ++e) mix((uint64_t)P.lcol[e]);
    return h;
}

bool same_structure(const Partition &P, int32_t a, int32_t b) {
    const int64_t ba = P.loc_ptr[a], bb = P.loc_ptr[b];
    const int64_t na = P.loc_ptr[a + 1] - ba, nb = P.loc_ptr[b + 1] - bb;
    if (na != nb) return false;
    const int64_t ea = P.lrp[ba], eb = P.lrp[bb];
    for (int64_t i = 0; i <= na; ++i)
        if (P.lrp[ba + i] - ea != P.lrp[bb + i] - eb) return false;
    return std::equal(P.lcol.begin() + ea, P.lcol.begin() + P.lrp[ba + na], P.lcol.begin() + eb);
}

int analyse(const Partition &P, int32_t k, int leaf, ClassSym &C, std::string &err) {
    const int64_t b = P.loc_ptr[k];
    const int32_t nk = (int32_t)(P.loc_ptr[k + 1] - b);
    if (nk >= 65535) { err = "subgraph too large for 16-bit local indices"; return VTM_ERR_PARTITION; }
    const int64_t e0 = P.lrp[b];
    LocalGraph g;
    g.nk = nk;
    g.ptr.assign(nk + 1, 0);
    for (int32_t i = 0; i < nk; ++i)
        for (int64_t e = P.lrp[b + i]; e < P.lrp[b + i + 1]; ++e)
            if (P.lcol[e] != i) g.adj.push_back(P.lcol[e]);
    for (int32_t i = 0, pos = 0; i < nk; ++i) {
        for (int64_t e = P.lrp[b + i]; e < P.lrp[b + i + 1]; ++e)
            if (P.lcol[e] != i) ++pos;
        g.ptr[i + 1] = pos;
    }
    g.has_coords = !P.coords.empty();
    g.xyz.assign(3 * (size_t)nk, 0.0);
    if (g.has_coords)
        for (int32_t i = 0; i < nk; ++i)
            for (int a = 0; a < P.dim; ++a) g.xyz[3 * i + a] = P.coords[P.loc_vtx[b + i] * P.dim + a];
    // ---- ordering and column blocks
    std::vector<std::vector<int32_t>> blocks;
    std::vector<int32_t> mark(nk, 0), all(nk);
    std::vector<double> coord(nk, 0.0);
    std::iota(all.begin(), all.end(), 0);
    int32_t tag = 0;
    dissect(g, all, std::max(1, leaf), mark, tag, coord, blocks);
    const int32_t nb = (int32_t)blocks.size();
    std::vector<int32_t> pos0(nk), bc0(nb + 1, 0), col2b(nk);
    {
        int32_t p = 0;
        for (int32_t s = 0; s < nb; ++s) {
            bc0[s] = p;
            for (int32_t v : blocks[s]) { pos0[v] = p; col2b[p] = s; ++p; }
        }
        bc0[nb] = p;
    }
    // ---- supernodal structure R_s and the assembly tree (original block order)
    std::vector<std::vector<int32_t>> R(nb), kids(nb);
    std::vector<int32_t> par(nb, -1), lev(nb, 0);
    for (int32_t s = 0; s < nb; ++s) {
        const int32_t last = bc0[s + 1] - 1;
        std::vector<int32_t> &r = R[s];
        for (int32_t v : blocks[s])
            for (int32_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e)
                if (pos0[g.adj[e]] > last) r.push_back(pos0[g.adj[e]]);
        for (int32_t c : kids[s])
            for (int32_t i : R[c])
                if (i > last) r.push_back(i);
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        for (int32_t c : kids[s]) lev[s] = std::max(lev[s], lev[c] + 1);
        if (!r.empty()) {
            par[s] = col2b[r[0]];
            kids[par[s]].push_back(s);
        }
    }
    // ---- renumber supernodes by (level, original order)
    std::vector<int32_t> order(nb);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return lev[a] < lev[c]; });
    std::vector<int32_t> newid(nb), newpos(nk);
    C = ClassSym();
    C.nk = nk;
    C.nsn = nb;
    C.sn_c0.resize(nb);
    C.sn_nc.resize(nb);
    {
        int32_t p = 0;
        for (int32_t t = 0; t < nb; ++t) {
            int32_t s = order[t];
            newid[s] = t;
            C.sn_c0[t] = p;
            C.sn_nc[t] = bc0[s + 1] - bc0[s];
            for (int32_t q = bc0[s]; q < bc0[s + 1]; ++q) newpos[q] = p++;
        }
    }
    C.perm.resize(nk);
    C.ipos.resize(nk);
    for (int32_t v = 0; v < nk; ++v) {
        C.ipos[v] = newpos[pos0[v]];
        C.perm[C.ipos[v]] = v;
    }
    C.sn_m.resize(nb);
    C.sn_parent.resize(nb);
    C.sn_level.resize(nb);
    std::vector<std::vector<int32_t>> Rn(nb);
    for (int32_t s = 0; s < nb; ++s) {
        int32_t t = newid[s];
        for (int32_t i : R[s]) Rn[t].push_back(newpos[i]);
        std::sort(Rn[t].begin(), Rn[t].end());
        C.sn_m[t] = (int32_t)Rn[t].size();
        C.sn_parent[t] = par[s] < 0 ? -1 : newid[par[s]];
        C.sn_level[t] = lev[s];
    }
    C.nlev = nb ? C.sn_level[nb - 1] + 1 : 0;
    C.lev_c0.assign(C.nlev + 1, nk);
    for (int32_t t = nb - 1; t >= 0; --t) C.lev_c0[C.sn_level[t]] = C.sn_c0[t];
    C.lev_c0[0] = 0;
    C.col_sn.resize(nk);
    for (int32_t t = 0; t < nb; ++t)
        for (int32_t q = 0; q < C.sn_nc[t]; ++q) C.col_sn[C.sn_c0[t] + q] = t;
    // ---- value / row-index / workspace layout
    C.sn_val.resize(nb);
    C.sn_ridx.resize(nb);
    C.sn_uoff.resize(nb);
    int64_t val = 0, ri = 0, uo = 0;
    C.nlower = 0;
    C.max_front = 0;
    for (int32_t t = 0; t < nb; ++t) {
        const int64_t nc = C.sn_nc[t], m = C.sn_m[t];
        C.sn_val[t] = (int32_t)val;
        C.sn_ridx[t] = (int32_t)ri;
        C.sn_uoff[t] = (int32_t)uo;
        val += nc * (nc + 1) / 2 + m * nc;  // packed: column j holds rows j .. nc + m - 1
        ri += m;
        uo += m * m;
        C.nlower += nc * (nc + 1) / 2 + m * nc;
        C.max_front = std::max<int32_t>(C.max_front, (int32_t)(nc + m));
        for (int32_t i : Rn[t]) C.ridx.push_back((uint16_t)i);
    }
    C.lev_maxf.assign(C.nlev + 1, 0);
    for (int32_t t = 0; t < nb; ++t)
        C.lev_maxf[C.sn_level[t]] = std::max<int32_t>(C.lev_maxf[C.sn_level[t]], C.sn_nc[t] + C.sn_m[t]);
    if (val > INT32_MAX || uo > INT32_MAX) { err = "local factor too large"; return VTM_ERR_PARTITION; }
    C.nval = val;
    C.ws_u = uo;
    // relative positions of R_s inside the parent's front (cols(p) then R_p)
    C.rel.resize(ri);
    for (int32_t t = 0; t < nb; ++t) {
        int32_t p = C.sn_parent[t];
        for (int32_t q = 0; q < C.sn_m[t]; ++q) {
            int32_t i = Rn[t][q];
            int32_t r;
            if (i >= C.sn_c0[p] && i < C.sn_c0[p] + C.sn_nc[p]) r = i - C.sn_c0[p];
            else {
                auto it = std::lower_bound(Rn[p].begin(), Rn[p].end(), i);
                if (it == Rn[p].end() || *it != i) { err = "assembly tree inconsistent"; return VTM_ERR_PARTITION; }
                r = C.sn_nc[p] + (int32_t)(it - Rn[p].begin());
            }
            C.rel[C.sn_ridx[t] + q] = (uint16_t)r;
        }
    }
    C.ch_ptr.assign(nb + 1, 0);
    for (int32_t t = 0; t < nb; ++t)
        if (C.sn_parent[t] >= 0) C.ch_ptr[C.sn_parent[t] + 1]++;
    for (int32_t t = 0; t < nb; ++t) C.ch_ptr[t + 1] += C.ch_ptr[t];
    C.ch_idx.resize(C.ch_ptr[nb]);
    {
        std::vector<int32_t> f(C.ch_ptr.begin(), C.ch_ptr.end() - 1);
        for (int32_t t = 0; t < nb; ++t)
            if (C.sn_parent[t] >= 0) C.ch_idx[f[C.sn_parent[t]]++] = t;
    }
    // forward-solve segments: row i receives L21_d[q, :] . y_d for every d with R_d[q] = i
    C.seg_ptr.assign(nk + 1, 0);
    for (int32_t t = 0; t < nb; ++t)
        for (int32_t i : Rn[t]) C.seg_ptr[i + 1]++;
    for (int32_t i = 0; i < nk; ++i) C.seg_ptr[i + 1] += C.seg_ptr[i];
    C.seg_off.resize(C.seg_ptr[nk]);
    C.seg_c0.resize(C.seg_ptr[nk]);
    C.seg_nc.resize(C.seg_ptr[nk]);
    C.seg_u.resize(C.seg_ptr[nk]);
    if (ri >= 65535) { err = "too many update entries for 16-bit indices"; return VTM_ERR_PARTITION; }
    C.u_sn.resize(ri);
    for (int32_t t = 0; t < nb; ++t)
        for (int32_t q = 0; q < C.sn_m[t]; ++q) C.u_sn[C.sn_ridx[t] + q] = (uint16_t)t;
    C.colrec.resize(4 * (size_t)nk);
    for (int32_t t = 0; t < nb; ++t)
        for (int32_t q = 0; q < C.sn_nc[t]; ++q) {
            int32_t *r = &C.colrec[4 * (size_t)(C.sn_c0[t] + q)];
            r[0] = C.sn_val[t];
            r[1] = (int32_t)(((uint32_t)C.sn_c0[t] << 16) | (uint32_t)C.sn_nc[t]);
            r[2] = (int32_t)(((uint32_t)q << 16) | (uint32_t)C.sn_m[t]);
            r[3] = C.sn_ridx[t];
        }
    C.urec.resize(4 * (size_t)ri);  // the colrec layout for row nc + q of the supernode (an update entry)
    for (int32_t t = 0; t < nb; ++t)
        for (int32_t q = 0; q < C.sn_m[t]; ++q) {
            int32_t *r = &C.urec[4 * (size_t)(C.sn_ridx[t] + q)];
            r[0] = C.sn_val[t];
            r[1] = (int32_t)(((uint32_t)C.sn_c0[t] << 16) | (uint32_t)C.sn_nc[t]);
            r[2] = (int32_t)(((uint32_t)(C.sn_nc[t] + q) << 16) | (uint32_t)C.sn_m[t]);
            r[3] = C.sn_ridx[t];
        }
    C.lev_u.assign(C.nlev + 1, (int32_t)ri);
    for (int32_t t = nb - 1; t >= 0; --t) C.lev_u[C.sn_level[t]] = C.sn_ridx[t];
    {
        std::vector<int32_t> f(C.seg_ptr.begin(), C.seg_ptr.end() - 1);
        for (int32_t t = 0; t < nb; ++t)
            for (int32_t q = 0; q < C.sn_m[t]; ++q) {
                int32_t i = Rn[t][q], s = f[i]++;
                C.seg_off[s] = C.sn_val[t] + C.sn_nc[t] * C.sn_nc[t] + q * C.sn_nc[t];
                C.seg_u[s] = (uint16_t)(C.sn_ridx[t] + q);
                C.seg_c0[s] = (uint16_t)C.sn_c0[t];
                C.seg_nc[s] = (uint16_t)C.sn_nc[t];
            }
    }
    // assembly scatter: lower entries of the local CSR into their column's front
    C.nnz_local = P.lrp[b + nk] - e0;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> sc(nb);
    for (int32_t li = 0; li < nk; ++li)
        for (int64_t e = P.lrp[b + li]; e < P.lrp[b + li + 1]; ++e) {
            const int32_t pi = C.ipos[li], pj = C.ipos[P.lcol[e]];
            if (pi < pj) continue;
            const int32_t t = C.col_sn[pj], c0 = C.sn_c0[t], nc = C.sn_nc[t], f = nc + C.sn_m[t];
            int32_t row;
            if (pi < c0 + nc) row = pi - c0;
            else {
                auto it = std::lower_bound(Rn[t].begin(), Rn[t].end(), pi);
                if (it == Rn[t].end() || *it != pi) { err = "front misses an entry"; return VTM_ERR_PARTITION; }
                row = nc + (int32_t)(it - Rn[t].begin());
            }
            sc[t].push_back({(int32_t)(e - e0), row * f + (pj - c0)});
        }
    // each front's list starts with the diagonals of its own columns in column order (every local row
    // holds its diagonal), so the assembly adds the port diagonal of column j to entry j
    C.sc_ptr.assign(nb + 1, 0);
    for (int32_t t = 0; t < nb; ++t) {
        const int32_t nc = C.sn_nc[t], f = nc + C.sn_m[t];
        std::vector<std::pair<int32_t, int32_t>> diag(nc, {-1, -1}), rest;
        for (auto &pr : sc[t]) {
            const int32_t row = pr.second / f, col = pr.second % f;
            if (row == col && row < nc) diag[row] = pr;
            else rest.push_back(pr);
        }
        for (int32_t j = 0; j < nc; ++j)
            if (diag[j].first < 0) { err = "front misses a diagonal entry"; return VTM_ERR_PARTITION; }
        C.sc_ptr[t + 1] = C.sc_ptr[t] + (int32_t)sc[t].size();
        for (auto &pr : diag) { C.sc_src.push_back(pr.first); C.sc_dst.push_back(pr.second); }
        for (auto &pr : rest) { C.sc_src.push_back(pr.first); C.sc_dst.push_back(pr.second); }
    }
    return VTM_OK;
}

}  // namespace

int build_symbolic(const Partition &P, int leaf, Symbolic &S, std::string &err) {
    S = Symbolic();
    S.sub_class.assign(P.nsub, -1);
    std::unordered_map<uint64_t, std::vector<int32_t>> seen;  // hash -> class ids
    std::vector<int32_t> rep;                                 // representative subgraph of each class
    for (int32_t k = 0; k < P.nsub; ++k) {
        uint64_t h = structure_hash(P, k);
        auto &cands = seen[h];
        int32_t found = -1;
        for (int32_t c : cands)
            if (same_structure(P, rep[c], k)) { found = c; break; }
        if (found < 0) {
            found = (int32_t)rep.size();
            rep.push_back(k);
            cands.push_back(found);
        }
        S.sub_class[k] = found;
    }
    S.classes.resize(rep.size());
    int rc = VTM_OK;
    std::string msg;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < (int32_t)rep.size(); ++c) {
        std::string e;
        int r = analyse(P, rep[c], leaf, S.classes[c], e);
        if (r) {
#pragma omp critical
            { rc = r; msg = e; }
        }
    }
    if (rc) err = msg;
    return rc;
}

}  // namespace vtm
