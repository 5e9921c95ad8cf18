// Dimensionless features of every VTL for the learned impedance model.
//
// The paper tunes the characteristic impedance by impedance matching (Section
// 7.1: Z near the input impedance of the ports).  The learned model predicts
// delta = ln(Z * a_vv), a multiplier over the diagonal rule, from local,
// scale-free quantities of the VTL's two ends (k, k2) at vertex v:
//   0,1  ln(d_k(v) / a_vv)                   min, max over the two ends
//   2,3  ln(inner_k(v) / a_vv + 1e-3)        branch weight towards interior vertices, min, max
//   4,5  ln n_k                               subgraph sizes, min, max
//   6,7  ln(#ports of k)                      min, max
//   8    ln(max(a_vv - sum_u |a_vu|, 0) / a_vv + 1e-6)   diagonal excess
//   9    ln |S(v)|                            children of v
//   10   ln(mean |a_uw| / a_vv)               over the edges within one hop of v's neighbours
//   11   ln(max |a_uw| / min |a_uw|)          same edges
//   12   ln(#subgraphs of v's system)         global scale: the best impedances grow with the number
//                                             of subgraphs information has to cross
// Every feature is invariant under scaling A by a positive constant.
#include <algorithm>
#include <cmath>

#include "vtm_internal.hpp"

namespace vtm {

void compute_features(const Csr &A, const Partition &P, std::vector<float> &out) {
    const int64_t nvtl = (int64_t)P.vtl_v.size();
    out.assign(nvtl * kNumFeatures, 0.f);
    std::vector<int64_t> nports(P.nsub), nsub_sys(std::max(P.nsys, 1), 0);
    for (int32_t k = 0; k < P.nsub; ++k) {
        nports[k] = P.port_ptr[k + 1] - P.port_ptr[k];
        ++nsub_sys[P.sub_sys.empty() ? 0 : P.sub_sys[k]];
    }
    auto nS = [&](int64_t v) { return P.s_ptr[v + 1] - P.s_ptr[v]; };
    auto end_stats = [&](int32_t k, int64_t v, double &dk, double &inner) {
        const int64_t *lv = P.loc_vtx.data() + P.loc_ptr[k];
        const int64_t nk = P.loc_ptr[k + 1] - P.loc_ptr[k];
        const int64_t li = std::lower_bound(lv, lv + nk, v) - lv;
        const int64_t row = P.loc_ptr[k] + li;
        dk = 0.0;
        inner = 0.0;
        for (int64_t e = P.lrp[row]; e < P.lrp[row + 1]; ++e) {
            const int32_t lj = P.lcol[e];
            if (lj == li) dk = P.lval[e];
            else if (nS(lv[lj]) == 1) inner += std::fabs(P.lval[e]);
        }
    };
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t l = 0; l < nvtl; ++l) {
        const int64_t v = P.vtl_v[l];
        const int32_t ka = P.vtl_k[l], kb = P.vtl_k2[l];
        const double avv = P.adiag[v];
        double da, ia, db, ib;
        end_stats(ka, v, da, ia);
        end_stats(kb, v, db, ib);
        const double na = (double)(P.loc_ptr[ka + 1] - P.loc_ptr[ka]), nb = (double)(P.loc_ptr[kb + 1] - P.loc_ptr[kb]);
        const double pa = (double)nports[ka], pb = (double)nports[kb];
        double absum = 0.0;
        double wsum = 0.0, wmax = 0.0, wmin = 1e300;
        int64_t wcnt = 0;
        for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e) {
            const int32_t u = A.ci[e];
            if (u == v) continue;
            absum += std::fabs(A.v[e]);
            for (int64_t f = A.rp[u]; f < A.rp[u + 1]; ++f) {
                if (A.ci[f] == u) continue;
                const double w = std::fabs(A.v[f]);
                wsum += w;
                wmax = std::max(wmax, w);
                wmin = std::min(wmin, w);
                ++wcnt;
            }
        }
        float *o = out.data() + l * kNumFeatures;
        const double f0 = std::log(da / avv), f1 = std::log(db / avv);
        const double g0 = std::log(ia / avv + 1e-3), g1 = std::log(ib / avv + 1e-3);
        o[0] = (float)std::min(f0, f1);
        o[1] = (float)std::max(f0, f1);
        o[2] = (float)std::min(g0, g1);
        o[3] = (float)std::max(g0, g1);
        o[4] = (float)std::log(std::min(na, nb));
        o[5] = (float)std::log(std::max(na, nb));
        o[6] = (float)std::log(std::min(pa, pb));
        o[7] = (float)std::log(std::max(pa, pb));
        o[8] = (float)std::log(std::max(avv - absum, 0.0) / avv + 1e-6);
        o[9] = (float)std::log((double)nS(v));
        o[10] = wcnt ? (float)std::log(wsum / wcnt / avv) : 0.f;
        o[11] = wcnt ? (float)std::log(wmax / wmin) : 0.f;
        o[12] = (float)std::log((double)nsub_sys[P.sub_sys.empty() ? 0 : P.sub_sys[ka]]);
    }
}

}  // namespace vtm
