// Electric Vertex Splitting on the host (Section 4 of Wei & Yang).
//
// Step 1 chooses the boundary through the membership S(v) of every vertex;
// step 2 gives vertex v one child per subgraph in S(v); step 3 splits vertex
// weights, edge weights (and, at solve time, sources); step 4 attaches ports,
// paired into virtual transmission lines (multilevel splitting, Fig. 7).
// Every floating-point split uses a fixed operation order so that the result
// is reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_set>

#include "vtm_internal.hpp"

namespace vtm {
namespace {

// splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators", 2014).
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        s += 0x9E3779B97F4A7C15ULL;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
};

struct Box {
    int32_t lo[3], hi[3];
};

int grid_membership(const vtm_partition_spec &sp, Partition &P, std::string &err) {
    const int32_t *d = sp.dims, *pa = sp.parts;
    if ((int64_t)d[0] * d[1] * d[2] != P.n) { err = "GRID dims do not match n"; return VTM_ERR_INVALID; }
    int32_t m[3];
    for (int a = 0; a < 3; ++a) {
        if (pa[a] < 1 || d[a] < 1) { err = "GRID parts/dims must be >= 1"; return VTM_ERR_INVALID; }
        m[a] = pa[a] == 1 ? d[a] : (d[a] % pa[a] == 0 ? d[a] / pa[a] : (d[a] - 1) / pa[a]);
        if (m[a] < 1 || (int64_t)(pa[a] - 1) * m[a] > d[a] - 1) { err = "GRID tiles too small"; return VTM_ERR_PARTITION; }
    }
    P.nsub = pa[0] * pa[1] * pa[2];
    P.s_ptr.assign(P.n + 1, 0);
    P.s_idx.clear();
    P.s_idx.reserve(P.n + P.n / 8);
    for (int64_t v = 0; v < P.n; ++v) {
        int32_t c[3] = {(int32_t)(v % d[0]), (int32_t)((v / d[0]) % d[1]), (int32_t)(v / ((int64_t)d[0] * d[1]))};
        int32_t t[3][2], nt[3];
        for (int a = 0; a < 3; ++a) {
            int32_t I = std::min(c[a] / m[a], pa[a] - 1);
            nt[a] = 0;
            if (I > 0 && c[a] == I * m[a]) t[a][nt[a]++] = I - 1;  // on the separator shared with tile I-1
            t[a][nt[a]++] = I;
        }
        for (int iz = 0; iz < nt[2]; ++iz)
            for (int iy = 0; iy < nt[1]; ++iy)
                for (int ix = 0; ix < nt[0]; ++ix) P.s_idx.push_back((t[2][iz] * pa[1] + t[1][iy]) * pa[0] + t[0][ix]);
        P.s_ptr[v + 1] = (int64_t)P.s_idx.size();
    }
    return VTM_OK;
}

// Leaf boxes of the seeded RCB of the vertex grid d (depth-first pre-order, explicit stack with
// the right child pushed first).  The cut percent is q = 49 + (splitmix64 mod 3).
int rcb_leaves(const int32_t *d, int levels, uint64_t seed, std::vector<Box> &leaves, std::string &err) {
    leaves.clear();
    leaves.reserve((size_t)1 << levels);
    SplitMix64 rng{seed};
    std::vector<std::pair<Box, int>> stack;
    Box root;
    for (int a = 0; a < 3; ++a) { root.lo[a] = 0; root.hi[a] = d[a] - 1; }
    stack.push_back({root, 0});
    while (!stack.empty()) {
        auto [b, depth] = stack.back();
        stack.pop_back();
        if (depth == levels) { leaves.push_back(b); continue; }
        int ax = 0;
        for (int a = 1; a < 3; ++a)
            if (b.hi[a] - b.lo[a] > b.hi[ax] - b.lo[ax]) ax = a;
        int32_t len = b.hi[ax] - b.lo[ax];
        if (len < 2) { err = "RCB box too thin to cut"; return VTM_ERR_PARTITION; }
        int32_t q = 49 + (int32_t)(rng.next() % 3);
        int32_t c = b.lo[ax] + (int32_t)(((int64_t)len * q + 50) / 100);
        Box l = b, r = b;
        l.hi[ax] = c;
        r.lo[ax] = c;
        stack.push_back({r, depth + 1});
        stack.push_back({l, depth + 1});
    }
    return VTM_OK;
}

constexpr int kRcbTries = 64;  // seeds seed, seed + 1, ... tried until every owned size is in bounds

int rcb_membership(const vtm_partition_spec &sp, Partition &P, std::string &err) {
    const int32_t *d = sp.dims;
    if ((int64_t)d[0] * d[1] * d[2] != P.n || sp.levels < 0 || sp.levels > 20) {
        err = "RCB dims/levels invalid";
        return VTM_ERR_INVALID;
    }
    std::vector<Box> leaves;
    std::vector<int32_t> cnt(P.n, 0);
    auto each = [&](const Box &b, auto &&fn) {
        for (int32_t z = b.lo[2]; z <= b.hi[2]; ++z)
            for (int32_t y = b.lo[1]; y <= b.hi[1]; ++y) {
                int64_t row = ((int64_t)z * d[1] + y) * d[0];
                for (int32_t x = b.lo[0]; x <= b.hi[0]; ++x) fn(row + x);
            }
    };
    std::string last;
    for (int t = 0; t < kRcbTries; ++t) {
        const uint64_t seed = sp.seed + (uint64_t)t;
        int rc = rcb_leaves(d, sp.levels, seed, leaves, err);
        if (rc) return rc;
        P.nsub = (int32_t)leaves.size();
        std::fill(cnt.begin(), cnt.end(), 0);
        for (const Box &b : leaves) each(b, [&](int64_t v) { cnt[v]++; });
        P.s_ptr.assign(P.n + 1, 0);
        for (int64_t v = 0; v < P.n; ++v) P.s_ptr[v + 1] = P.s_ptr[v] + cnt[v];
        bool ok = true;
        for (int32_t k = 0; k < P.nsub && ok; ++k) {
            double own = 0.0;  // ascending vertex order
            each(leaves[k], [&](int64_t v) { own += 1.0 / (double)(P.s_ptr[v + 1] - P.s_ptr[v]); });
            if (own < sp.min_size || own > sp.max_size) {
                ok = false;
                last = "RCB box " + std::to_string(k) + " owned size " + std::to_string(own) + " outside bounds";
            }
        }
        if (!ok) continue;
        P.s_idx.assign(P.s_ptr[P.n], 0);
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int32_t k = 0; k < P.nsub; ++k) each(leaves[k], [&](int64_t v) { P.s_idx[P.s_ptr[v] + cnt[v]++] = k; });
        P.rcb_seed = seed;
        return VTM_OK;
    }
    err = last + " for seeds " + std::to_string(sp.seed) + " .. " + std::to_string(sp.seed + kRcbTries - 1);
    return VTM_ERR_PARTITION;
}

// Parts whose owned vertices fall apart: a coordinate cut of a graph can leave a few vertices in a
// part that they touch only through other parts.  Such a piece reaches the rest of its system only
// through VTLs and holds a slowly decaying wave mode.  Parts in increasing id: the owned vertices of
// part k are split into connected components (edges of A between vertices owned by k), the largest
// stays (ties: the one with the smallest vertex), and every other component goes to the part it
// shares the most edges with (ties: the smallest id); a component with no edge leaving the part (a
// component of A) stays.  A moved component is connected to its new part, so a part processed
// earlier stays connected.
void connect_parts(const Csr &A, std::vector<int32_t> &owner, int32_t nsub) {
    const int64_t n = A.n;
    std::vector<std::vector<int64_t>> members(nsub);
    for (int64_t v = 0; v < n; ++v) members[owner[v]].push_back(v);
    std::vector<int32_t> comp(n, -1);
    std::vector<int64_t> queue, start;  // vertices by component (BFS order), component starts
    std::vector<std::pair<int32_t, int32_t>> cnt;
    for (int32_t k = 0; k < nsub; ++k) {
        std::vector<int64_t> &mv = members[k];
        std::sort(mv.begin(), mv.end());
        queue.clear();
        start.clear();
        int32_t nc = 0;
        for (const int64_t s : mv) {
            if (comp[s] >= 0) continue;
            start.push_back((int64_t)queue.size());
            comp[s] = nc;
            queue.push_back(s);
            for (size_t h = (size_t)start.back(); h < queue.size(); ++h) {
                const int64_t v = queue[h];
                for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e) {
                    const int32_t u = A.ci[e];
                    if (owner[u] == k && comp[u] < 0) {
                        comp[u] = nc;
                        queue.push_back(u);
                    }
                }
            }
            ++nc;
        }
        start.push_back((int64_t)queue.size());
        if (nc > 1) {
            int32_t keep = 0;
            for (int32_t c = 1; c < nc; ++c)
                if (start[c + 1] - start[c] > start[keep + 1] - start[keep]) keep = c;
            for (int32_t c = 0; c < nc; ++c) {
                if (c == keep) continue;
                cnt.clear();
                for (int64_t i = start[c]; i < start[c + 1]; ++i) {
                    const int64_t v = queue[i];
                    for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e) {
                        const int32_t q = owner[A.ci[e]];
                        if (q != k) cnt.push_back({q, 1});
                    }
                }
                if (cnt.empty()) continue;
                std::sort(cnt.begin(), cnt.end());
                int32_t best = -1, best_n = 0;
                for (size_t i = 0; i < cnt.size();) {
                    size_t j = i;
                    while (j < cnt.size() && cnt[j].first == cnt[i].first) ++j;
                    if ((int32_t)(j - i) > best_n) { best_n = (int32_t)(j - i); best = cnt[i].first; }
                    i = j;
                }
                for (int64_t i = start[c]; i < start[c + 1]; ++i) {
                    owner[queue[i]] = best;
                    members[best].push_back(queue[i]);
                }
            }
        }
        for (const int64_t v : queue) comp[v] = -1;
        std::vector<int64_t>().swap(mv);
    }
}

int graph_membership(const vtm_partition_spec &sp, const Csr &A, Partition &P, std::string &err) {
    if (!sp.coords || sp.dim < 1 || sp.dim > 3 || sp.nblocks < 1 || !sp.block_start || !sp.block_count ||
        !sp.block_parts) {
        err = "GRAPH needs coords and blocks";
        return VTM_ERR_INVALID;
    }
    const int dim = sp.dim;
    const double *X = sp.coords;
    std::vector<int32_t> owner(P.n, -1);
    int32_t next = 0;
    std::vector<int64_t> vs;
    struct Task { int64_t b, e; int32_t np; };
    for (int32_t blk = 0; blk < sp.nblocks; ++blk) {
        int64_t s0 = sp.block_start[blk], cnt = sp.block_count[blk];
        int32_t np = sp.block_parts[blk];
        if (np < 1 || cnt < np || s0 < 0 || s0 + cnt > P.n) { err = "GRAPH block invalid"; return VTM_ERR_PARTITION; }
        vs.resize(cnt);
        std::iota(vs.begin(), vs.end(), s0);
        // depth-first, left part first: explicit stack with the right task pushed first
        std::vector<Task> st{{0, cnt, np}};
        while (!st.empty()) {
            Task t = st.back();
            st.pop_back();
            if (t.np == 1) {
                int32_t id = next++;
                for (int64_t i = t.b; i < t.e; ++i) owner[vs[i]] = id;
                continue;
            }
            int ax = 0;
            double best = -1.0;
            for (int a = 0; a < dim; ++a) {
                double lo = X[vs[t.b] * dim + a], hi = lo;
                for (int64_t i = t.b + 1; i < t.e; ++i) {
                    double c = X[vs[i] * dim + a];
                    lo = std::min(lo, c);
                    hi = std::max(hi, c);
                }
                if (hi - lo > best) { best = hi - lo; ax = a; }
            }
            std::sort(vs.begin() + t.b, vs.begin() + t.e, [&](int64_t u, int64_t v) {
                double cu = X[u * dim + ax], cv = X[v * dim + ax];
                return cu < cv || (cu == cv && u < v);
            });
            int32_t nl = t.np / 2;
            int64_t cut = ((t.e - t.b) * (int64_t)nl) / t.np;
            st.push_back({t.b + cut, t.e, t.np - nl});
            st.push_back({t.b, t.b + cut, nl});
        }
    }
    for (int64_t v = 0; v < P.n; ++v)
        if (owner[v] < 0) { err = "GRAPH blocks do not cover all vertices"; return VTM_ERR_PARTITION; }
    connect_parts(A, owner, next);
    P.nsub = next;
    P.s_ptr.assign(P.n + 1, 0);
    P.s_idx.clear();
    std::vector<int32_t> tmp;
    for (int64_t v = 0; v < P.n; ++v) {
        tmp.clear();
        tmp.push_back(owner[v]);
        for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e) {
            int32_t u = A.ci[e];
            if (u != v && owner[u] > owner[v]) tmp.push_back(owner[u]);
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        P.s_idx.insert(P.s_idx.end(), tmp.begin(), tmp.end());
        P.s_ptr[v + 1] = (int64_t)P.s_idx.size();
    }
    return VTM_OK;
}

inline bool contains(const int32_t *a, int64_t na, int32_t x) { return std::binary_search(a, a + na, x); }

inline int intersect_count(const int32_t *a, int64_t na, const int32_t *b, int64_t nb) {
    int c = 0;
    int64_t i = 0, j = 0;
    while (i < na && j < nb) {
        if (a[i] == b[j]) { ++c; ++i; ++j; }
        else if (a[i] < b[j]) ++i;
        else ++j;
    }
    return c;
}

}  // namespace

int build_partition(const Csr &A, const vtm_partition_spec &sp, Partition &P, std::string &err) {
    P = Partition();
    P.n = A.n;
    const int64_t n = A.n;
    // ---- validate the CSR: sorted columns, explicit positive diagonal, finite, symmetric
    P.adiag.assign(n, 0.0);
    for (int64_t v = 0; v < n; ++v) {
        bool diag = false;
        for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e) {
            int32_t u = A.ci[e];
            if (u < 0 || u >= n || !std::isfinite(A.v[e]) || (e > A.rp[v] && u <= A.ci[e - 1])) {
                err = "row " + std::to_string(v) + ": bad column order/index or non-finite value";
                return VTM_ERR_INVALID;
            }
            if (u == v) {
                diag = true;
                P.adiag[v] = A.v[e];
                if (!(A.v[e] > 0.0)) { err = "non-positive diagonal at " + std::to_string(v); return VTM_ERR_INVALID; }
            } else {
                const int32_t *b = A.ci.data() + A.rp[u], *e2 = A.ci.data() + A.rp[u + 1];
                const int32_t *f = std::lower_bound(b, e2, (int32_t)v);
                if (f == e2 || *f != v || A.v[A.rp[u] + (f - b)] != A.v[e]) {
                    err = "matrix is not symmetric at (" + std::to_string(v) + "," + std::to_string(u) + ")";
                    return VTM_ERR_INVALID;
                }
            }
        }
        if (!diag) { err = "missing diagonal at " + std::to_string(v); return VTM_ERR_INVALID; }
    }
    // ---- step 1: membership
    int rc = VTM_OK;
    switch (sp.kind) {
        case VTM_PART_GRID: rc = grid_membership(sp, P, err); break;
        case VTM_PART_RCB: rc = rcb_membership(sp, P, err); break;
        case VTM_PART_GRAPH: rc = graph_membership(sp, A, P, err); break;
        case VTM_PART_USER:
            if (!sp.s_ptr || !sp.s_idx || sp.user_nsub < 1) { err = "USER needs s_ptr, s_idx, nsub"; return VTM_ERR_INVALID; }
            P.nsub = sp.user_nsub;
            P.s_ptr.assign(sp.s_ptr, sp.s_ptr + n + 1);
            P.s_idx.assign(sp.s_idx, sp.s_idx + sp.s_ptr[n]);
            for (int64_t v = 0; v < n; ++v) {
                if (P.s_ptr[v + 1] <= P.s_ptr[v]) { err = "vertex without subgraph"; return VTM_ERR_PARTITION; }
                for (int64_t i = P.s_ptr[v]; i < P.s_ptr[v + 1]; ++i)
                    if (P.s_idx[i] < 0 || P.s_idx[i] >= P.nsub || (i > P.s_ptr[v] && P.s_idx[i] <= P.s_idx[i - 1])) {
                        err = "USER membership not sorted/in range";
                        return VTM_ERR_PARTITION;
                    }
            }
            break;
        default: err = "unknown partition kind"; return VTM_ERR_INVALID;
    }
    if (rc) return rc;
    auto S = [&](int64_t v) { return P.s_idx.data() + P.s_ptr[v]; };
    auto nS = [&](int64_t v) { return P.s_ptr[v + 1] - P.s_ptr[v]; };
    // every edge must lie inside some subgraph
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e) {
            int32_t u = A.ci[e];
            if (u != v && !intersect_count(S(v), nS(v), S(u), nS(u))) {
                err = "edge (" + std::to_string(v) + "," + std::to_string(u) + ") is not inside any subgraph";
                return VTM_ERR_PARTITION;
            }
        }
    // ---- step 2: children; local vertex lists ascending
    const int32_t nsub = P.nsub;
    P.loc_ptr.assign(nsub + 1, 0);
    for (int64_t i = 0; i < P.s_ptr[n]; ++i) P.loc_ptr[P.s_idx[i] + 1]++;
    for (int32_t k = 0; k < nsub; ++k) {
        if (P.loc_ptr[k + 1] == 0) { err = "subgraph " + std::to_string(k) + " is empty"; return VTM_ERR_PARTITION; }
        P.loc_ptr[k + 1] += P.loc_ptr[k];
    }
    const int64_t nsplit = P.loc_ptr[nsub];
    P.loc_vtx.assign(nsplit, 0);
    {
        std::vector<int64_t> fill(P.loc_ptr.begin(), P.loc_ptr.end() - 1);
        for (int64_t v = 0; v < n; ++v)
            for (int64_t i = P.s_ptr[v]; i < P.s_ptr[v + 1]; ++i) P.loc_vtx[fill[P.s_idx[i]]++] = v;
    }
    // ---- step 3: split weights into the pieces A~_k
    P.lrp.assign(nsplit + 1, 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t k = 0; k < nsub; ++k)
        for (int64_t li = P.loc_ptr[k]; li < P.loc_ptr[k + 1]; ++li) {
            int64_t v = P.loc_vtx[li], c = 0;
            for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e)
                if (A.ci[e] == v || contains(S(A.ci[e]), nS(A.ci[e]), k)) ++c;
            P.lrp[li + 1] = c;
        }
    for (int64_t li = 0; li < nsplit; ++li) P.lrp[li + 1] += P.lrp[li];
    P.lcol.assign(P.lrp[nsplit], 0);
    P.lval.assign(P.lrp[nsplit], 0.0);
    const bool equal_rule = sp.split_rule == VTM_SPLIT_EQUAL;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t k = 0; k < nsub; ++k) {
        const int64_t *lv = P.loc_vtx.data() + P.loc_ptr[k];
        const int64_t nk = P.loc_ptr[k + 1] - P.loc_ptr[k];
        for (int64_t i = 0; i < nk; ++i) {
            const int64_t v = lv[i];
            double absum = 0.0;  // sum of |a_vu| over all branches of v, column order
            for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e)
                if (A.ci[e] != v) absum += std::fabs(A.v[e]);
            double share = 0.0;  // sum of this child's branch magnitudes, column order
            int64_t out = P.lrp[P.loc_ptr[k] + i], dpos = -1;
            for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e) {
                const int32_t u = A.ci[e];
                if (u == v) { dpos = out; P.lcol[out++] = (int32_t)i; continue; }
                if (!contains(S(u), nS(u), k)) continue;
                const int64_t lu = std::lower_bound(lv, lv + nk, (int64_t)u) - lv;
                const double w = A.v[e] / (double)intersect_count(S(v), nS(v), S(u), nS(u));
                P.lcol[out] = (int32_t)lu;
                P.lval[out++] = w;
                share += std::fabs(w);
            }
            const double m = (double)nS(v), avv = P.adiag[v];
            P.lval[dpos] = nS(v) == 1 ? avv : (equal_rule ? avv / m : share + (avv - absum) / m);
        }
    }
    // ---- step 4: VTLs between children (multilevel splitting) and ports
    std::unordered_set<uint64_t> face;
    for (int64_t v = 0; v < n; ++v)
        if (nS(v) == 2) face.insert(((uint64_t)(uint32_t)S(v)[0] << 32) | (uint32_t)S(v)[1]);
    for (int64_t v = 0; v < n; ++v) {
        const int m = (int)nS(v);
        if (m < 2) continue;
        const int32_t *sv = S(v);
        std::vector<std::pair<int, int>> pairs, all;
        for (int a = 0; a < m; ++a)
            for (int b = a + 1; b < m; ++b) {
                all.push_back({a, b});
                if (sp.topology != VTM_TOPO_COMPLETE && face.count(((uint64_t)(uint32_t)sv[a] << 32) | (uint32_t)sv[b]))
                    pairs.push_back({a, b});
            }
        if (sp.topology == VTM_TOPO_COMPLETE) pairs = all;
        else {
            // union-find over the children of v
            std::vector<int> par(m);
            std::iota(par.begin(), par.end(), 0);
            auto find = [&](int x) { while (par[x] != x) x = par[x] = par[par[x]]; return x; };
            for (auto &pr : pairs) par[find(pr.first)] = find(pr.second);
            bool connected = true;
            for (int a = 1; a < m; ++a) connected &= find(a) == find(0);
            if (!connected) pairs = all;
        }
        if (sp.topology == VTM_TOPO_TREE) {
            // repeated binary splits: one VTL per split, a spanning tree of the pairs above (greedy in
            // (k, k') order), so that no cycle of VTLs meets at v
            std::vector<int> root(m);
            std::iota(root.begin(), root.end(), 0);
            auto top = [&](int x) { while (root[x] != x) x = root[x] = root[root[x]]; return x; };
            std::vector<std::pair<int, int>> tree;
            for (auto &pr : pairs) {
                const int ra = top(pr.first), rb = top(pr.second);
                if (ra == rb) continue;
                root[rb] = ra;
                tree.push_back(pr);
            }
            pairs.swap(tree);
        }
        for (auto &pr : pairs) {
            P.vtl_v.push_back(v);
            P.vtl_k.push_back(sv[pr.first]);
            P.vtl_k2.push_back(sv[pr.second]);
        }
    }
    const int64_t nvtl = (int64_t)P.vtl_v.size(), nports = 2 * nvtl;
    // ports of subgraph k sorted by (v, other end); twin = the other end of the same VTL
    struct PortRec { int64_t v; int32_t other; int64_t vtl; };
    std::vector<std::vector<PortRec>> per(nsub);
    for (int64_t l = 0; l < nvtl; ++l) {
        per[P.vtl_k[l]].push_back({P.vtl_v[l], P.vtl_k2[l], l});
        per[P.vtl_k2[l]].push_back({P.vtl_v[l], P.vtl_k[l], l});
    }
    P.port_ptr.assign(nsub + 1, 0);
    for (int32_t k = 0; k < nsub; ++k) P.port_ptr[k + 1] = P.port_ptr[k] + (int64_t)per[k].size();
    P.port_v.resize(nports);
    P.port_other.resize(nports);
    P.port_vtl.resize(nports);
    P.port_twin.resize(nports);
    P.port_lidx.resize(nports);
    std::vector<int64_t> ends(2 * nvtl, -1);
    for (int32_t k = 0; k < nsub; ++k) {
        auto &vec = per[k];
        std::sort(vec.begin(), vec.end(), [](const PortRec &a, const PortRec &b) {
            return a.v < b.v || (a.v == b.v && a.other < b.other);
        });
        const int64_t *lv = P.loc_vtx.data() + P.loc_ptr[k];
        const int64_t nk = P.loc_ptr[k + 1] - P.loc_ptr[k];
        for (size_t i = 0; i < vec.size(); ++i) {
            int64_t p = P.port_ptr[k] + (int64_t)i;
            P.port_v[p] = vec[i].v;
            P.port_other[p] = vec[i].other;
            P.port_vtl[p] = vec[i].vtl;
            P.port_lidx[p] = (int32_t)(std::lower_bound(lv, lv + nk, vec[i].v) - lv);
            int64_t &slot = ends[2 * vec[i].vtl + (P.vtl_k[vec[i].vtl] == k ? 0 : 1)];
            slot = p;
        }
    }
    for (int64_t l = 0; l < nvtl; ++l) {
        P.port_twin[ends[2 * l]] = ends[2 * l + 1];
        P.port_twin[ends[2 * l + 1]] = ends[2 * l];
    }
    // diagonal impedance rule
    P.zdiag.resize(nvtl);
    for (int64_t l = 0; l < nvtl; ++l) P.zdiag[l] = 1.0 / P.adiag[P.vtl_v[l]];
    // coordinates for the local orderings
    if (sp.kind == VTM_PART_GRID || sp.kind == VTM_PART_RCB) {
        P.dim = 3;
        P.coords.resize(3 * n);
        for (int64_t v = 0; v < n; ++v) {
            P.coords[3 * v + 0] = (double)(v % sp.dims[0]);
            P.coords[3 * v + 1] = (double)((v / sp.dims[0]) % sp.dims[1]);
            P.coords[3 * v + 2] = (double)(v / ((int64_t)sp.dims[0] * sp.dims[1]));
        }
    } else if (sp.coords && sp.dim >= 1 && sp.dim <= 3) {
        P.dim = sp.dim;
        P.coords.assign(sp.coords, sp.coords + n * sp.dim);
    }
    // systems
    if (sp.nsys > 1) {
        if (!sp.sys_ptr || sp.sys_ptr[0] != 0 || sp.sys_ptr[sp.nsys] != n) { err = "sys_ptr invalid"; return VTM_ERR_INVALID; }
        P.nsys = sp.nsys;
        P.sys_ptr.assign(sp.sys_ptr, sp.sys_ptr + sp.nsys + 1);
    } else {
        P.nsys = 1;
        P.sys_ptr = {0, n};
    }
    P.sub_sys.assign(nsub, 0);
    for (int32_t k = 0; k < nsub; ++k) {
        int64_t v0 = P.loc_vtx[P.loc_ptr[k]], v1 = P.loc_vtx[P.loc_ptr[k + 1] - 1];
        int32_t s0 = (int32_t)(std::upper_bound(P.sys_ptr.begin(), P.sys_ptr.end(), v0) - P.sys_ptr.begin()) - 1;
        int32_t s1 = (int32_t)(std::upper_bound(P.sys_ptr.begin(), P.sys_ptr.end(), v1) - P.sys_ptr.begin()) - 1;
        if (s0 != s1) { err = "a subgraph spans two systems"; return VTM_ERR_PARTITION; }
        P.sub_sys[k] = s0;
    }
    return VTM_OK;
}

}  // namespace vtm
