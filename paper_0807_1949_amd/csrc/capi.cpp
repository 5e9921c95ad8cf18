// C ABI of libvtm: handle, EVS partition upload, setup (Z + factorisation) and
// the VTM solve loop (Table 1 of Wei & Yang) with FP64 or FP32 + FP64
// iterative refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "mlp.hpp"
#include "vtm.h"
#include "vtm_debug.h"
#include "vtm_internal.hpp"

namespace vtm {
std::string &last_error_ref() {
    static thread_local std::string err;
    return err;
}
}  // namespace vtm

namespace {


vtm_status fail(vtm_status code, const std::string &msg) {
    vtm::last_error_ref() = msg;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            if (e_ == hipErrorOutOfMemory) return fail(VTM_ERR_OOM, std::string(#expr) + ": out of memory"); \
            return fail(VTM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                                 \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const { return reinterpret_cast<T *>(p); }
};

// HIP events released on every return path.
struct Events {
    hipEvent_t e[5] = {};
    int n = 0;
    hipError_t create(int count) {
        for (; n < count; ++n) {
            hipError_t r = hipEventCreate(&e[n]);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    hipEvent_t operator[](int i) const { return e[i]; }
    ~Events() {
        for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]);
    }
};

}  // namespace

struct vtm_ctx {
    vtm_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    vtm::Csr A;
    vtm::Partition P;
    vtm::Symbolic S;
    bool partitioned = false, set_up = false;
    int32_t max_nk = 0, max_front = 0;
    int64_t nsplit = 0, nports = 0, total_val = 0, total_ws = 0, total_lower = 0;
    std::vector<DevBuf *> all;
    // symbolic (class level)
    DevBuf d_segu, d_usn, d_levu, d_colrec, d_urec;
    // port-reduced sweeps
    DevBuf d_goff, d_G64, d_G32, d_cport, d_gorder, d_portpg;
    int32_t max_p = 0, npg = 0, max_np = 0;
    // per system: packed G entries, port vertices, ports, stored factor entries, split entries
    std::vector<double> sys_g, sys_pg, sys_ports, sys_lower, sys_split;
    int32_t persist_R = -1, persist_ng = -1;
    bool persist_fits = false;
    int64_t total_g = 0;   // stored entries of all packed G_k
    bool plan_in_order = false;  // every subgraph's plan order is its port-vertex order (G_k by k_gram)
    double total_pp = 0;   // sum of p_k^2 (entries of the full G_k)
    bool have_green = false;
    bool have_y = false;  // the set-up kept the Y blocks (FP64 workspace, FP32 copy when sweeping in FP32)
    bool yb_ok = false;   // yb holds L^{-1} b~ of the current source split
    bool have_y32 = false;  // d_gws32 is written by the factorisation
    bool gws_clean = false; // the port fronts in d_gws are all zero
    // column plan of the multifrontal Green's-function computation (built on first use)
    DevBuf d_gsn, d_gbase, d_gwso, d_gidoff, d_gperm, d_gws, d_levmaxf;
    int plan_state = 0;  // 0 not built, 1 ready, -1 not applicable (fall back to per-column solves)
    int64_t gws_total = 0;
    std::vector<int32_t> h_pgptr, h_pgbeg, h_pgcnt;
    std::vector<uint16_t> h_pgpos;
    int32_t max_nu = 0;
    DevBuf d_cls, d_lev, d_colsn, d_snc0, d_snnc, d_snm, d_snval, d_snridx, d_snuoff, d_ridx, d_rel, d_chptr, d_chidx,
        d_segptr, d_segoff, d_segc0, d_segnc, d_scptr, d_scdst;
    // subgraph level
    DevBuf d_subcls, d_subval, d_subx, d_subaval, d_subws, d_pgptr, d_pgpos, d_pgbeg, d_pgcnt, d_portptr;
    // maps, matrix, ports
    DevBuf d_fvtx, d_fmul, d_cpptr, d_cpidx, d_rp, d_ci, d_v, d_aval, d_twin, d_portvtl, d_chunkrow, d_chunksys,
        d_syschunk, d_subsys, d_active;
    bool mask_on = false;          // sweeps and test solves skip converged systems (batched solves)
    DevBuf d_sublist;              // subgraphs of the systems still sweeping, largest G_k first
    std::vector<int32_t> h_gorder, h_sublist;
    bool list_on = false;          // launches cover d_sublist only (h_sublist.size() workgroups)
    DevBuf d_rlist;                // subgraphs of the systems whose refinement restarts at this test
    std::vector<int32_t> h_rlist;
    bool rl_on = false;            // launches cover d_rlist only (restart of some systems)
    int32_t *active_host = nullptr;  // pinned per-system flags of the done mask
    size_t active_cap = 0;
    int32_t *rowflag_host = nullptr;  // pinned per-system row moves of a test (see launch_sys_rows)
    size_t rowflag_cap = 0;
    DevBuf d_rowflag;
    uint64_t setup_id = 0;         // unique id of the last vtm_setup (batch solves rebuild when one changes)
    vtm_ctx *batch = nullptr;      // concatenation of handles for vtm_batch_solve (owned)
    std::vector<uint64_t> batch_key;
    // coupled VTLs: the local pieces carry the off-diagonal entries of Z_j^{-1}; the EVS pieces are kept
    bool coupled = false;
    std::vector<int64_t> lrp0;
    std::vector<int32_t> lcol0;
    std::vector<double> lval0;
    DevBuf d_cplptr, d_cpltw, d_cply64, d_cply32;
    int32_t nchunks = 0;
    // setup products
    DevBuf d_z, d_invz64, d_invz32, d_vals64, d_vals32, d_status;
    // learned impedance model
    DevBuf d_zparams, d_feat, d_avvl, d_pred;
    DevBuf d_ws;  // factorisation workspace (update matrices, large fronts, port diagonal), kept between set-ups
    DevBuf d_gws32, d_yb;  // FP32 copy of the Y blocks; y_b = L^{-1} b~ per RHS group
    bool model_loaded = false, feats_ready = false, feats_on_dev = false;
    std::vector<float> feats;
    // solve state
    DevBuf d_o[2], d_bsplit, d_xloc, d_x, d_xt, d_r, d_rt, d_b, d_part, d_relres;
    int cur = 0;
    int32_t wave_nrhs = 0, wave_R = 1;
    // captured sweep batches, one per starting wave buffer
    struct SweepGraph {
        hipGraphExec_t exec = nullptr;
        int64_t count = 0;
        int32_t R = 0, ng = 0, threads = 0, variant = 0;
        const void *ptrs[8] = {};
        int32_t nlaunch = 0;
    } graphs[2];
    void drop_graphs() {
        for (auto &g : graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            g = SweepGraph();
        }
    }
    bool waves_zero = true;
    // persistent port-reduced sweeps: tagged wave words, abort flag, next sweep tag
    DevBuf d_tw, d_abort;
    int32_t tag = 1;
    int64_t persist_launches = 0;  // persistent launches of the current solve or run
    double *relres_host = nullptr;  // pinned copy of the residual norms of a test
    size_t relres_cap = 0;
    hipEvent_t ev_test = nullptr;   // completion of a test's residual copy (polled)
    bool abort_pending = false;
    vtm_stats stats{};
    bool trace = false;  // VTM_TRACE set: one line per convergence test on stderr
    int32_t ncu = 0;     // compute units of the device

    vtm_ctx() {
        DevBuf *list[] = {&d_cls, &d_lev, &d_colsn, &d_snc0, &d_snnc, &d_snm, &d_snval, &d_snridx, &d_snuoff, &d_ridx,
                          &d_rel, &d_chptr, &d_chidx, &d_segptr, &d_segoff, &d_segc0, &d_segnc, &d_scptr,
                          &d_scdst, &d_subcls, &d_subval, &d_subx, &d_subaval, &d_subws, &d_pgptr, &d_pgpos,
                          &d_pgbeg, &d_pgcnt, &d_portptr, &d_fvtx, &d_fmul, &d_cpptr, &d_cpidx, &d_rp, &d_ci, &d_v, &d_aval,
                          &d_twin, &d_portvtl, &d_chunkrow, &d_chunksys, &d_syschunk, &d_subsys, &d_active, &d_sublist, &d_rlist, &d_rowflag, &d_cplptr, &d_cpltw, &d_cply64, &d_cply32, &d_z, &d_invz64, &d_invz32,
                          &d_vals64, &d_vals32, &d_status, &d_segu, &d_usn, &d_levu, &d_colrec, &d_urec, &d_goff, &d_G64, &d_G32, &d_cport, &d_gorder, &d_portpg, &d_gsn, &d_gbase, &d_gwso, &d_gidoff, &d_gperm, &d_gws, &d_levmaxf, &d_tw, &d_abort, &d_zparams, &d_feat, &d_avvl, &d_pred, &d_ws, &d_gws32, &d_yb, &d_o[0], &d_o[1], &d_bsplit, &d_xloc, &d_x, &d_xt, &d_r,
                          &d_rt, &d_b, &d_part, &d_relres};
        for (DevBuf *b : list) all.push_back(b);
    }
    bool host_only() const { return opt.device < 0; }
    ~vtm_ctx() {
        if (host_only()) return;
        (void)hipSetDevice(opt.device);
        drop_graphs();
        for (DevBuf *b : all) b->release();
        delete batch;
        if (relres_host) (void)hipHostFree(relres_host);
        if (active_host) (void)hipHostFree(active_host);
        if (rowflag_host) (void)hipHostFree(rowflag_host);
        if (ev_test) (void)hipEventDestroy(ev_test);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    bool fp32() const { return opt.precision == VTM_FP32_IR; }
    size_t tsize() const { return fp32() ? sizeof(float) : sizeof(double); }
};

namespace {

hipError_t ensure(DevBuf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return hipSuccess;
    b.release();
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.bytes = bytes;
    return e;
}

template <typename T>
hipError_t upload(DevBuf &b, const std::vector<T> &v, hipStream_t st) {
    hipError_t e = ensure(b, sizeof(T) * std::max<size_t>(v.size(), 1));
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st);
}

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

vtm::DevSym dev_sym(vtm_ctx *h) {
    vtm::DevSym s;
    s.cls = h->d_cls.as<vtm::ClassDev>();
    s.lev_c0 = h->d_lev.as<int32_t>();
    s.col_sn = h->d_colsn.as<int32_t>();
    s.lev_maxf = h->d_levmaxf.as<int32_t>();
    s.sn_c0 = h->d_snc0.as<int32_t>();
    s.sn_nc = h->d_snnc.as<int32_t>();
    s.sn_m = h->d_snm.as<int32_t>();
    s.sn_val = h->d_snval.as<int32_t>();
    s.sn_ridx = h->d_snridx.as<int32_t>();
    s.sn_uoff = h->d_snuoff.as<int32_t>();
    s.ridx = h->d_ridx.as<uint16_t>();
    s.rel = h->d_rel.as<uint16_t>();
    s.ch_ptr = h->d_chptr.as<int32_t>();
    s.ch_idx = h->d_chidx.as<int32_t>();
    s.seg_ptr = h->d_segptr.as<int32_t>();
    s.seg_off = h->d_segoff.as<int32_t>();
    s.seg_c0 = h->d_segc0.as<uint16_t>();
    s.seg_nc = h->d_segnc.as<uint16_t>();
    s.seg_u = h->d_segu.as<uint16_t>();
    s.colrec = h->d_colrec.as<int32_t>();
    s.urec = h->d_urec.as<int32_t>();
    s.u_sn = h->d_usn.as<uint16_t>();
    s.lev_u = h->d_levu.as<int32_t>();
    s.sc_ptr = h->d_scptr.as<int32_t>();
    s.sc_dst = h->d_scdst.as<int32_t>();
    return s;
}

vtm::DevSub dev_sub(vtm_ctx *h) {
    vtm::DevSub d;
    d.cls = h->d_subcls.as<int32_t>();
    d.val = h->d_subval.as<int64_t>();
    d.x = h->d_subx.as<int64_t>();
    d.aval = h->d_subaval.as<int64_t>();
    d.ws = h->d_subws.as<int64_t>();
    d.pg_ptr = h->d_pgptr.as<int32_t>();
    d.pg_pos = h->d_pgpos.as<uint16_t>();
    d.pg_beg = h->d_pgbeg.as<int32_t>();
    d.pg_cnt = h->d_pgcnt.as<int32_t>();
    d.port_ptr = h->d_portptr.as<int32_t>();
    d.port_pg = h->d_portpg.as<uint16_t>();
    d.gorder = h->d_gorder.as<int32_t>();
    d.sub_sys = h->d_subsys.as<int32_t>();
    d.active = h->mask_on ? h->d_active.as<int32_t>() : nullptr;
    d.cpl_ptr = h->coupled ? h->d_cplptr.as<int32_t>() : nullptr;
    d.cpl_tw = h->d_cpltw.as<int32_t>();
    d.cpl_y64 = h->d_cply64.as<double>();
    d.cpl_y32 = h->d_cply32.as<float>();
    d.sub_list = h->rl_on ? h->d_rlist.as<int32_t>() : h->mask_on && h->list_on ? h->d_sublist.as<int32_t>() : nullptr;
    return d;
}

// Workgroups of a launch over the subgraphs: the restart list, the active list under the done mask,
// else all.
int32_t nsub_launch(const vtm_ctx *h) {
    return h->rl_on ? (int32_t)h->h_rlist.size() : h->mask_on && h->list_on ? (int32_t)h->h_sublist.size() : h->P.nsub;
}

// Column plan of the port Green's functions (computed inside k_factor).  Ports are sorted by the
// postorder of their supernode; the ports below supernode s then form the range [lo_s, lo_s + w_s),
// its own ports the tail of it.  Workspace per supernode: port front (nc + m) x w_s, then Y_s (nc x w_s).
// Postorder number of every supernode of a class's assembly tree, and the smallest postorder number
// in its subtree (first): the subtree of s is the range [first[s], post[s]].
void sn_postorder(const vtm::ClassSym &C, std::vector<int32_t> &post, std::vector<int32_t> &first) {
    std::vector<std::vector<int32_t>> ch(C.nsn);
    std::vector<int32_t> roots;
    for (int32_t s = 0; s < C.nsn; ++s) (C.sn_parent[s] < 0 ? roots : ch[C.sn_parent[s]]).push_back(s);
    post.assign(C.nsn, 0);
    first.assign(C.nsn, 0);
    int32_t cnt = 0;
    std::vector<std::pair<int32_t, size_t>> stack;  // (supernode, next child)
    for (int32_t r : roots) {
        stack.push_back({r, 0});
        first[r] = cnt;
        while (!stack.empty()) {
            auto &top = stack.back();
            if (top.second < ch[top.first].size()) {
                const int32_t q = ch[top.first][top.second++];
                first[q] = cnt;
                stack.push_back({q, 0});
            } else {
                post[top.first] = cnt++;
                stack.pop_back();
            }
        }
    }
}

vtm_status build_green_plan(vtm_ctx *h) {
    const vtm::Partition &P = h->P;
    const vtm::Symbolic &S = h->S;
    const int32_t nsub = P.nsub;
    std::vector<std::vector<int32_t>> post(S.classes.size()), first(S.classes.size());
    for (size_t c = 0; c < S.classes.size(); ++c) sn_postorder(S.classes[c], post[c], first[c]);
    std::vector<int4> sn;
    std::vector<int32_t> base(nsub + 1, 0), idoff(h->npg, 0);
    std::vector<uint16_t> perm(h->npg, 0);
    std::vector<int64_t> wso(nsub + 1, 0);
    bool in_order = true;
    for (int32_t k = 0; k < nsub; ++k) {
        const int32_t c = S.sub_class[k];
        const vtm::ClassSym &C = S.classes[c];
        const int32_t pg0 = h->h_pgptr[k], p = h->h_pgptr[k + 1] - pg0;
        std::vector<int32_t> key(p), order(p);
        for (int32_t j = 0; j < p; ++j) {
            key[j] = post[c][C.col_sn[h->h_pgpos[pg0 + j]]];
            order[j] = j;
        }
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
        std::vector<int32_t> ks(p);
        for (int32_t a = 0; a < p; ++a) ks[a] = key[order[a]];
        std::vector<int32_t> lo(C.nsn), w(C.nsn);
        std::vector<int64_t> fo(C.nsn);
        int64_t off = 0;
        for (int32_t s = 0; s < C.nsn; ++s) {
            lo[s] = (int32_t)(std::lower_bound(ks.begin(), ks.end(), first[c][s]) - ks.begin());
            w[s] = (int32_t)(std::upper_bound(ks.begin(), ks.end(), post[c][s]) - ks.begin()) - lo[s];
            off = (off + 3) & ~(int64_t)3;  // regions start on 4 entries (16-byte rows of the FP32 Y blocks)
            fo[s] = off;
            off += (int64_t)(2 * C.sn_nc[s] + C.sn_m[s]) * w[s];
        }
        if (off >= ((int64_t)1 << 31)) {
            h->plan_state = -1;
            return VTM_OK;
        }
        base[k] = (int32_t)sn.size();
        for (int32_t s = 0; s < C.nsn; ++s) {
            const int32_t par = C.sn_parent[s];
            sn.push_back(int4{(int32_t)fo[s], lo[s] | (w[s] << 16), par < 0 ? 0 : (int32_t)fo[par],
                              par < 0 ? 0 : (lo[par] | (w[par] << 16))});
        }
        for (int32_t a = 0; a < p; ++a) {
            const int32_t j = order[a], pos = h->h_pgpos[pg0 + j], s = C.col_sn[pos];
            in_order = in_order && j == a;
            perm[pg0 + a] = (uint16_t)j;
            idoff[pg0 + a] = (int32_t)(fo[s] + (int64_t)(pos - C.sn_c0[s]) * w[s] + (a - lo[s]));
        }
        wso[k + 1] = wso[k] + ((off + 3) & ~(int64_t)3);
    }
    base[nsub] = (int32_t)sn.size();
    h->gws_total = wso[nsub];
    hipStream_t st = h->stream;
    HIP_TRY(upload(h->d_gsn, sn, st));
    HIP_TRY(upload(h->d_gbase, base, st));
    HIP_TRY(upload(h->d_gwso, wso, st));
    HIP_TRY(upload(h->d_gidoff, idoff, st));
    HIP_TRY(upload(h->d_gperm, perm, st));
    HIP_TRY(hipStreamSynchronize(st));
    h->plan_in_order = in_order;
    h->plan_state = 1;
    return VTM_OK;
}

vtm::DevGreen dev_green(vtm_ctx *h, bool on) {
    vtm::DevGreen g{};
    if (!on) return g;
    g.sn = h->d_gsn.as<int4>();
    g.base = h->d_gbase.as<int32_t>();
    g.wso = h->d_gwso.as<int64_t>();
    g.idoff = h->d_gidoff.as<int32_t>();
    g.perm = h->d_gperm.as<uint16_t>();
    g.ws = h->d_gws.as<double>();
    g.ws32 = h->have_y32 ? h->d_gws32.as<float>() : nullptr;
    return g;
}

vtm::DevMaps dev_maps(vtm_ctx *h) {
    vtm::DevMaps m;
    m.fvtx = h->d_fvtx.as<int32_t>();
    m.fmul = h->d_fmul.as<int32_t>();
    m.cp_ptr = h->d_cpptr.as<int64_t>();
    m.cp_idx = h->d_cpidx.as<int32_t>();
    return m;
}

void host_sizes(vtm_ctx *h) {
    h->max_nk = 0;
    h->max_front = 0;
    for (const vtm::ClassSym &C : h->S.classes) {
        h->max_nk = std::max(h->max_nk, C.nk);
        h->max_front = std::max(h->max_front, C.max_front);
    }
    h->total_lower = 0;
    for (int32_t k = 0; k < h->P.nsub; ++k) h->total_lower += h->S.classes[h->S.sub_class[k]].nlower;
    h->nsplit = h->P.loc_ptr[h->P.nsub];
    h->nports = (int64_t)h->P.port_v.size();
}

vtm_status upload_partition(vtm_ctx *h) {
    const vtm::Partition &P = h->P;
    const vtm::Symbolic &S = h->S;
    hipStream_t st = h->stream;
    // ---- class arrays
    std::vector<vtm::ClassDev> cls;
    std::vector<int32_t> lev, colsn, snc0, snnc, snm, snval, snridx, snuoff, chptr, chidx, segptr, segoff, scptr,
        scdst;
    std::vector<uint16_t> ridx, rel, segc0, segnc, segu, usn;
    std::vector<int32_t> levu, colrec, urec, levmaxf;
    h->max_nk = 0;
    h->max_front = 0;
    h->max_nu = 0;
    for (const vtm::ClassSym &C : S.classes) {
        vtm::ClassDev d{};
        d.nk = C.nk;
        d.nsn = C.nsn;
        d.nlev = C.nlev;
        d.max_front = C.max_front;
        d.o_lev = (int32_t)lev.size();
        d.o_sn = (int32_t)snc0.size();
        d.o_snp = (int32_t)chptr.size();
        d.o_col = (int32_t)colsn.size();
        d.o_colp = (int32_t)segptr.size();
        d.o_ridx = (int32_t)ridx.size();
        d.o_seg = (int32_t)segoff.size();
        d.o_sc = (int32_t)scdst.size();
        d.o_chi = (int32_t)chidx.size();
        d.nval = C.nval;
        d.ws_u = C.ws_u;
        d.nu = (int32_t)C.ridx.size();
        h->max_nu = std::max(h->max_nu, d.nu);
        cls.push_back(d);
        levu.insert(levu.end(), C.lev_u.begin(), C.lev_u.end());
        segu.insert(segu.end(), C.seg_u.begin(), C.seg_u.end());
        usn.insert(usn.end(), C.u_sn.begin(), C.u_sn.end());
        colrec.insert(colrec.end(), C.colrec.begin(), C.colrec.end());
        urec.insert(urec.end(), C.urec.begin(), C.urec.end());
        lev.insert(lev.end(), C.lev_c0.begin(), C.lev_c0.end());
        levmaxf.insert(levmaxf.end(), C.lev_maxf.begin(), C.lev_maxf.end());
        colsn.insert(colsn.end(), C.col_sn.begin(), C.col_sn.end());
        snc0.insert(snc0.end(), C.sn_c0.begin(), C.sn_c0.end());
        snnc.insert(snnc.end(), C.sn_nc.begin(), C.sn_nc.end());
        snm.insert(snm.end(), C.sn_m.begin(), C.sn_m.end());
        snval.insert(snval.end(), C.sn_val.begin(), C.sn_val.end());
        snridx.insert(snridx.end(), C.sn_ridx.begin(), C.sn_ridx.end());
        snuoff.insert(snuoff.end(), C.sn_uoff.begin(), C.sn_uoff.end());
        chptr.insert(chptr.end(), C.ch_ptr.begin(), C.ch_ptr.end());
        scptr.insert(scptr.end(), C.sc_ptr.begin(), C.sc_ptr.end());
        chidx.insert(chidx.end(), C.ch_idx.begin(), C.ch_idx.end());
        segptr.insert(segptr.end(), C.seg_ptr.begin(), C.seg_ptr.end());
        segoff.insert(segoff.end(), C.seg_off.begin(), C.seg_off.end());
        segc0.insert(segc0.end(), C.seg_c0.begin(), C.seg_c0.end());
        segnc.insert(segnc.end(), C.seg_nc.begin(), C.seg_nc.end());
        ridx.insert(ridx.end(), C.ridx.begin(), C.ridx.end());
        rel.insert(rel.end(), C.rel.begin(), C.rel.end());
        scdst.insert(scdst.end(), C.sc_dst.begin(), C.sc_dst.end());
        h->max_nk = std::max(h->max_nk, C.nk);
        h->max_front = std::max(h->max_front, C.max_front);
        // ch_ptr/sc_ptr share o_snp: both have nsn + 1 entries per class
    }
    // ---- subgraph arrays
    const int32_t nsub = P.nsub;
    std::vector<int32_t> subcls(nsub), pgptr(nsub + 1, 0), pgbeg, pgcnt;
    std::vector<int64_t> subval(nsub), subx(nsub), subaval(nsub), subws(nsub);
    std::vector<uint16_t> pgpos, portpg(P.port_v.size());
    std::vector<double> afront;  // lower entries of every local matrix in the order of its class's scatter list
    int64_t vo = 0, wo = 0;
    h->total_lower = 0;
    std::vector<std::vector<int32_t>> post(S.classes.size());
    {
        std::vector<int32_t> first;
        for (size_t c = 0; c < S.classes.size(); ++c) sn_postorder(S.classes[c], post[c], first);
    }
    struct PortGroup {
        int32_t key, beg, cnt;
        uint16_t pos;
    };
    std::vector<PortGroup> groups;
    for (int32_t k = 0; k < nsub; ++k) {
        const int32_t c = S.sub_class[k];
        const vtm::ClassSym &C = S.classes[c];
        subcls[k] = c;
        subval[k] = vo;
        vo += C.nval;
        h->total_lower += C.nlower;
        subx[k] = P.loc_ptr[k];
        subaval[k] = (int64_t)afront.size();
        for (const int32_t src : C.sc_src) afront.push_back(P.lval[P.lrp[P.loc_ptr[k]] + src]);
        subws[k] = wo;
        wo += C.ws_u + (int64_t)C.max_front * C.max_front + ((C.nk + 1) & ~1);  // updates, front, port diagonal
        // the port vertices (groups of ports at one vertex) in the postorder of the supernodes holding
        // them: the ports below any supernode are then contiguous, so that the G_k block that a
        // supernode's Y_s^T Y_s adds to is a contiguous block of the packed G_k (coalesced adds)
        groups.clear();
        for (int64_t p = P.port_ptr[k]; p < P.port_ptr[k + 1];) {
            int64_t q = p;
            while (q < P.port_ptr[k + 1] && P.port_v[q] == P.port_v[p]) ++q;
            const uint16_t pos = (uint16_t)C.ipos[P.port_lidx[p]];
            groups.push_back(PortGroup{post[c][C.col_sn[pos]], (int32_t)p, (int32_t)(q - p), pos});
            p = q;
        }
        std::stable_sort(groups.begin(), groups.end(),
                         [](const PortGroup &a, const PortGroup &b) { return a.key < b.key; });
        for (const PortGroup &g : groups) {
            for (int32_t t = g.beg; t < g.beg + g.cnt; ++t) portpg[t] = (uint16_t)(pgpos.size() - pgptr[k]);
            pgpos.push_back(g.pos);
            pgbeg.push_back(g.beg);
            pgcnt.push_back(g.cnt);
        }
        pgptr[k + 1] = (int32_t)pgpos.size();
    }
    h->total_val = vo;
    h->total_ws = wo;
    h->h_pgptr = pgptr;
    h->h_pgpos = pgpos;
    h->h_pgbeg = pgbeg;
    h->h_pgcnt = pgcnt;
    h->plan_state = 0;
    h->gws_clean = false;
    {
        std::vector<int64_t> goff(nsub + 1, 0);
        h->max_p = 0;
        h->total_pp = 0;
        h->persist_R = h->persist_ng = -1;
        for (int32_t k = 0; k < nsub; ++k) {
            // packed symmetric G_k: lower block triangle of 16 x 16 blocks
            const int64_t p = pgptr[k + 1] - pgptr[k], nb = (p + 15) / 16;
            goff[k + 1] = goff[k] + nb * (nb + 1) / 2 * 256;
            h->total_pp += (double)p * (double)p;
            h->max_p = std::max<int32_t>(h->max_p, (int32_t)p);
        }
        h->total_g = goff[nsub];
        h->npg = pgptr[nsub];
        h->sys_g.assign(P.nsys, 0.0);
        h->sys_pg.assign(P.nsys, 0.0);
        h->sys_ports.assign(P.nsys, 0.0);
        h->sys_lower.assign(P.nsys, 0.0);
        h->sys_split.assign(P.nsys, 0.0);
        for (int32_t k = 0; k < nsub; ++k) {
            const int32_t y = P.sub_sys[k];
            h->sys_g[y] += (double)(goff[k + 1] - goff[k]);
            h->sys_pg[y] += (double)(pgptr[k + 1] - pgptr[k]);
            h->sys_ports[y] += (double)(P.port_ptr[k + 1] - P.port_ptr[k]);
            h->sys_lower[y] += (double)S.classes[S.sub_class[k]].nlower;
            h->sys_split[y] += (double)(P.loc_ptr[k + 1] - P.loc_ptr[k]);
        }
        HIP_TRY(upload(h->d_goff, goff, st));
        // launch order of the port-reduced sweep: largest G_k first (ties by subgraph id)
        std::vector<int32_t> gorder(nsub);
        for (int32_t k = 0; k < nsub; ++k) gorder[k] = k;
        std::stable_sort(gorder.begin(), gorder.end(), [&](int32_t a, int32_t b) {
            return goff[a + 1] - goff[a] > goff[b + 1] - goff[b];
        });
        HIP_TRY(upload(h->d_gorder, gorder, st));
        h->h_gorder = gorder;
    }
    h->nsplit = P.loc_ptr[nsub];
    h->nports = (int64_t)P.port_v.size();
    // ---- split/merge maps (factor order inside every subgraph)
    std::vector<int32_t> fvtx(h->nsplit), fmul(h->nsplit), cpidx(P.s_ptr[P.n]);
    std::vector<int64_t> cpfill(P.s_ptr.begin(), P.s_ptr.end() - 1);
    for (int32_t k = 0; k < nsub; ++k) {
        const vtm::ClassSym &C = S.classes[S.sub_class[k]];
        const int64_t b = P.loc_ptr[k];
        for (int32_t i = 0; i < C.nk; ++i) {
            const int64_t v = P.loc_vtx[b + i];
            const int64_t e = b + C.ipos[i];
            cpidx[cpfill[v]++] = (int32_t)e;
        }
        for (int32_t pos = 0; pos < C.nk; ++pos) {
            const int64_t v = P.loc_vtx[b + C.perm[pos]];
            fvtx[b + pos] = (int32_t)v;
            fmul[b + pos] = (int32_t)(P.s_ptr[v + 1] - P.s_ptr[v]);
        }
    }
    std::vector<int32_t> twin(h->nports), portvtl(h->nports);
    for (int64_t p = 0; p < h->nports; ++p) {
        twin[p] = (int32_t)P.port_twin[p];
        portvtl[p] = (int32_t)P.port_vtl[p];
    }
    // residual chunks: contiguous row ranges inside one system
    std::vector<int64_t> chunkrow;
    std::vector<int32_t> chunksys, syschunk(P.nsys + 1, 0);
    const int64_t CH = 256;  // one row per thread of the residual kernel
    for (int32_t s = 0; s < P.nsys; ++s) {
        for (int64_t r = P.sys_ptr[s]; r < P.sys_ptr[s + 1]; r += CH) {
            chunkrow.push_back(r);
            chunksys.push_back(s);
        }
        syschunk[s + 1] = (int32_t)chunkrow.size();
    }
    chunkrow.push_back(P.n);
    h->nchunks = (int32_t)chunksys.size();

#define UP(buf, vec) HIP_TRY(upload(h->buf, vec, st))
    UP(d_cls, cls); UP(d_lev, lev); UP(d_levmaxf, levmaxf); UP(d_colsn, colsn); UP(d_snc0, snc0); UP(d_snnc, snnc); UP(d_snm, snm);
    UP(d_snval, snval); UP(d_snridx, snridx); UP(d_snuoff, snuoff); UP(d_ridx, ridx); UP(d_rel, rel);
    UP(d_chptr, chptr); UP(d_chidx, chidx); UP(d_segptr, segptr); UP(d_segoff, segoff); UP(d_segc0, segc0);
    UP(d_segnc, segnc); UP(d_segu, segu); UP(d_usn, usn); UP(d_levu, levu); UP(d_colrec, colrec); UP(d_urec, urec); UP(d_scptr, scptr); UP(d_scdst, scdst);
    UP(d_subcls, subcls); UP(d_subval, subval); UP(d_subx, subx); UP(d_subaval, subaval); UP(d_subws, subws);
    UP(d_pgptr, pgptr); UP(d_pgpos, pgpos); UP(d_pgbeg, pgbeg); UP(d_pgcnt, pgcnt); UP(d_portpg, portpg);
    {
        std::vector<int32_t> portptr(nsub + 1);
        h->max_np = 0;
        for (int32_t k = 0; k <= nsub; ++k) portptr[k] = (int32_t)P.port_ptr[k];
        for (int32_t k = 0; k < nsub; ++k) h->max_np = std::max(h->max_np, portptr[k + 1] - portptr[k]);
        UP(d_portptr, portptr);
    }
    UP(d_fvtx, fvtx); UP(d_fmul, fmul); UP(d_cpptr, P.s_ptr); UP(d_cpidx, cpidx);
    UP(d_rp, h->A.rp); UP(d_ci, h->A.ci); UP(d_v, h->A.v); UP(d_aval, afront);
    UP(d_twin, twin); UP(d_portvtl, portvtl); UP(d_chunkrow, chunkrow); UP(d_chunksys, chunksys);
    UP(d_syschunk, syschunk); UP(d_subsys, P.sub_sys);
#undef UP
    HIP_TRY(hipStreamSynchronize(st));
    return VTM_OK;
}

int32_t pick_R(vtm_ctx *h, int32_t nrhs) {
    if (h->opt.rhs_per_block > 0) return h->opt.rhs_per_block;
    int32_t want = 1;
    while (want < nrhs && want < 8) want *= 2;
    while (want > 1 && 2 * h->tsize() * (size_t)h->max_nk * want > 96 * 1024) want /= 2;
    return want;
}

// Bytes of one wave buffer: ng x nports x R values and one spare, rounded to 16 (one fill kernel).
template <typename T>
size_t wave_bytes(const vtm_ctx *h, int32_t nrhs, int32_t R) {
    const int32_t ng = (nrhs + R - 1) / R;
    return (sizeof(T) * ((size_t)ng * h->nports * R + 1) + 15) & ~(size_t)15;
}

template <typename T>
vtm_status ensure_waves(vtm_ctx *h, int32_t nrhs) {
    const int32_t R = pick_R(h, nrhs);
    const size_t bytes = wave_bytes<T>(h, nrhs, R);
    if (h->wave_nrhs != nrhs || h->wave_R != R || !h->d_o[0].p) {
        HIP_TRY(ensure(h->d_o[0], bytes));
        HIP_TRY(ensure(h->d_o[1], bytes));
        HIP_TRY(hipMemsetAsync(h->d_o[0].p, 0, bytes, h->stream));
        HIP_TRY(hipMemsetAsync(h->d_o[1].p, 0, bytes, h->stream));
        h->wave_nrhs = nrhs;
        h->wave_R = R;
        h->cur = 0;
        h->waves_zero = true;
    }
    return VTM_OK;
}

template <typename T>
vtm_status zero_waves(vtm_ctx *h) {
    if (h->waves_zero) return VTM_OK;  // nothing has written the waves since they were cleared
    HIP_TRY(hipMemsetAsync(h->d_o[h->cur].p, 0, wave_bytes<T>(h, h->wave_nrhs, h->wave_R), h->stream));
    h->waves_zero = true;
    return VTM_OK;
}

// A caller's column-major n x nrhs block (host or device, leading dimension ld) into row-interleaved
// device rows (stride vec_stride(nrhs)); a host block passes through the device buffer staging
// (column-major, at least n x nrhs), which the stream order keeps until the conversion has read it.
vtm_status to_rows(vtm_ctx *h, const double *src, int64_t ld, int64_t n, int32_t nrhs, double *dst, double *staging) {
    const int32_t S = vtm::vec_stride(nrhs);
    if (!is_device_ptr(src)) {
        HIP_TRY(hipMemcpy2DAsync(staging, sizeof(double) * n, src, sizeof(double) * ld, sizeof(double) * n, nrhs,
                                 hipMemcpyHostToDevice, h->stream));
        src = staging;
        ld = n;
    }
    vtm::launch_to_rows(src, ld, n, nrhs, S, dst, h->stream);
    return VTM_OK;
}

// Row-interleaved device rows into a caller's column-major block (host or device), through staging
// for a host destination.
vtm_status from_rows(vtm_ctx *h, const double *src, int64_t n, int32_t nrhs, double *dst, int64_t ld, double *staging) {
    const int32_t S = vtm::vec_stride(nrhs);
    if (is_device_ptr(dst)) {
        vtm::launch_from_rows(src, S, n, nrhs, dst, ld, h->stream);
        return VTM_OK;
    }
    vtm::launch_from_rows(src, S, n, nrhs, staging, n, h->stream);
    HIP_TRY(hipMemcpy2DAsync(dst, sizeof(double) * ld, staging, sizeof(double) * n, sizeof(double) * n, nrhs,
                             hipMemcpyDeviceToHost, h->stream));
    return VTM_OK;
}

// Stage b (host or device) into the handle's FP64 device copy (row-interleaved; after alloc_solve, whose
// residual buffer stages a host b).
vtm_status stage_b(vtm_ctx *h, const double *b, int32_t nrhs, int64_t ldb) {
    const int64_t n = h->P.n;
    HIP_TRY(ensure(h->d_b, sizeof(double) * (size_t)n * vtm::vec_stride(nrhs)));
    return to_rows(h, b, ldb, n, nrhs, h->d_b.as<double>(), h->d_rt.as<double>());
}

// After a stream synchronisation: did a persistent launch since the last check give up on a wait?
// fetched is the flag as copied with the residual norms, or -1 (then it is read here).
vtm_status check_abort(vtm_ctx *h, int fetched = -1) {
    if (!h->abort_pending) return VTM_OK;
    h->abort_pending = false;
    int32_t flag = fetched;
    if (flag < 0) {
        HIP_TRY(hipMemcpyAsync(&flag, h->d_abort.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    if (flag) {
        HIP_TRY(hipMemsetAsync(h->d_abort.p, 0, sizeof(int32_t), h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        return fail(VTM_ERR_HIP, "persistent sweep: a wave exchange wait timed out");
    }
    return VTM_OK;
}

// x (row-interleaved src, one of the two iterate buffers) to the caller; the residual buffer stages a
// host destination.
vtm_status write_x(vtm_ctx *h, const double *src, double *x, int32_t nrhs, int64_t ldx) {
    vtm_status rc;
    if ((rc = from_rows(h, src, h->P.n, nrhs, x, ldx, h->d_r.as<double>()))) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return check_abort(h);
}

template <typename T>
T *vals_of(vtm_ctx *h) {
    if constexpr (sizeof(T) == 4) return h->d_vals32.as<T>();
    else return h->d_vals64.as<T>();
}
template <typename T>
T *green_of(vtm_ctx *h) {
    if constexpr (sizeof(T) == 4) return h->d_G32.as<T>();
    else return h->d_G64.as<T>();
}
template <typename T>
T *invz_of(vtm_ctx *h) {
    if constexpr (sizeof(T) == 4) return h->d_invz32.as<T>();
    else return h->d_invz64.as<T>();
}

// Port-reduced sweeps when the Green's functions exist and move no more than twice the factor's bytes.
// Port-reduced sweeps by default when the packed G_k hold at most this many times the stored factor
// entries: the G stream runs near HBM bandwidth while the substitution is bound by its level chain
// (3D Poisson, 4096 boxes, 8 RHS: G 4.1x the factor and still 2x faster per sweep).
constexpr double kGreenRatio = 8.0;

bool use_schur(vtm_ctx *h) {
    if (!h->have_green || h->coupled) return false;
    // the port vectors of a workgroup (R right-hand sides) must fit in LDS
    if (vtm::schur_lds_bytes(h->tsize(), h->max_p, h->max_np, std::max(1, h->wave_R), h->opt.sweep_waves) > vtm::kMaxLds) return false;
    if (h->opt.sweep_mode == 2) return true;
    if (h->opt.sweep_mode == 1) return false;
    return (double)h->total_g <= kGreenRatio * (double)h->total_lower;
}

int32_t sweep_variant(vtm_ctx *h) {
    const int32_t v = h->opt.sweep_variant;
    if (v == 1 || v == 2) return v - 1;
    // default: gather update entries when they fit in LDS with the vectors
    return h->tsize() * (size_t)h->wave_R * (2 * (size_t)h->max_nk + h->max_nu) <= 96 * 1024 ? 1 : 0;
}

int32_t sweep_threads(vtm_ctx *h) {
    const int32_t t = h->opt.sweep_threads;
    return t >= 64 && t <= 512 && t % 64 == 0 ? t : 256;
}

// Sweeps on the current waves; the last one stores the local solutions.  Batches of two or more
// sweeps are captured once into a HIP graph per starting wave buffer and replayed.
// Persistent port-reduced sweeps need FP32, every workgroup resident at once and each wave's G
// blocks in registers.
bool persistent_ok(vtm_ctx *h, int32_t R, int32_t ng) {
    if (!h->fp32() || h->opt.persistent == 1 || !use_schur(h)) return false;
    if (R != 1 && R != 2) return false;  // wider groups spill the on-chip G blocks to scratch
    if (h->max_p > vtm::persist_max_p()) return false;  // G_k rows held in registers
    if (vtm::persist_lds_bytes(h->max_p, h->max_np, R) > vtm::kMaxLds) return false;
    if (h->persist_R != R || h->persist_ng != ng) {
        int64_t resident = 0;
        if (vtm::persist_capacity(h->max_p, h->max_np, R, &resident) != hipSuccess) {
            (void)hipGetLastError();
            resident = 0;
        }
        h->persist_R = R;
        h->persist_ng = ng;
        h->persist_fits = (int64_t)h->P.nsub * ng <= resident;
    }
    return h->persist_fits;
}

constexpr int32_t kSpinLimit = 1 << 20;  // polls of one wave word before a persistent launch gives up

template <typename T>
vtm_status run_sweeps_dev(vtm_ctx *h, int64_t count) {
    if (count <= 0) return VTM_OK;
    const vtm::DevSym S = dev_sym(h);
    const vtm::DevSub D = dev_sub(h);
    const int32_t R = h->wave_R, ng = (h->wave_nrhs + R - 1) / R, nt = sweep_threads(h);
    HIP_TRY(vtm::prepare_sweep<T>(h->max_nk, h->max_nu, sweep_variant(h), R));
    const bool schur = use_schur(h);
    // waves per subgraph of the streaming sweep: the option, else two when the subgraphs still
    // sweeping would leave most CUs idle (the tail of a batch), so that each G_k streams on two waves
    int32_t W = h->opt.sweep_waves;
    if (schur && W == 0 && h->ncu > 0 && (int64_t)nsub_launch(h) * ng < 2 * (int64_t)h->ncu &&
        vtm::schur_lds_bytes(h->tsize(), h->max_p, h->max_np, R, 2) <= vtm::kMaxLds)
        W = 2;
    if (schur) HIP_TRY(vtm::prepare_schur<T>(h->max_p, h->max_np, R, W));
    if constexpr (std::is_same<T, float>::value) {
        if (schur && persistent_ok(h, R, ng)) {
            const int64_t nw = (int64_t)ng * h->nports * R;
            const void *tw_before = h->d_tw.p;
            HIP_TRY(ensure(h->d_tw, sizeof(unsigned long long) * (2 * nw + 2)));
            // tag 0 is never awaited (tags start at 1): a new buffer holds no word a launch could take
            if (h->d_tw.p != tw_before) HIP_TRY(hipMemsetAsync(h->d_tw.p, 0, h->d_tw.bytes, h->stream));
            if (!h->d_abort.p) {
                HIP_TRY(ensure(h->d_abort, sizeof(int32_t) * 2));
                HIP_TRY(hipMemsetAsync(h->d_abort.p, 0, sizeof(int32_t), h->stream));
            }
            bool refused = false;
            for (int64_t left = count; left > 0;) {
                const int32_t nsw = (int32_t)std::min<int64_t>(left, 1 << 20);
                if (h->tag > (1 << 29)) h->tag = 1;
                const hipError_t e = vtm::launch_schur_persist(
                    D, h->P.nsub, ng, R, h->max_p, h->max_np, h->npg, h->nports, green_of<float>(h),
                    h->d_goff.as<int64_t>(), h->d_cport.as<float>(), h->d_twin.as<int32_t>(), invz_of<float>(h),
                    h->d_tw.as<unsigned long long>(), h->d_o[0].as<float>(), h->d_o[1].as<float>(), h->tag, nsw,
                    h->cur, h->opt.spin_limit > 0 ? h->opt.spin_limit : kSpinLimit, h->d_abort.as<int32_t>(),
                    h->stream);
                if (e != hipSuccess && left == count) {  // not co-resident after all: per-sweep launches
                    (void)hipGetLastError();
                    h->persist_fits = false;
                    refused = true;
                    break;
                }
                HIP_TRY(e);
                h->tag += nsw + 2;
                h->cur ^= (int)(nsw & 1);
                ++h->persist_launches;
                left -= nsw;
            }
            if (refused) goto per_sweep;
            // the flag comes to the host with the next residual norms, or is read at the caller's next
            // synchronisation (check_abort); it stays set until then
            h->abort_pending = true;
            h->waves_zero = false;
            h->stats.persistent = 1;
            return VTM_OK;
        }
    }
per_sweep:
    auto launch = [&](int cur, bool last) {
        if (schur)
            vtm::launch_schur<T>(D, nsub_launch(h), ng, R, W, h->max_p, h->max_np, h->npg, h->nports, green_of<T>(h),
                                 h->d_goff.as<int64_t>(), h->d_cport.as<T>(), h->d_twin.as<int32_t>(), invz_of<T>(h),
                                 h->d_o[cur].as<T>(), h->d_o[1 - cur].as<T>(), h->stream);
        else
            vtm::launch_sweep<T>(S, D, nsub_launch(h), h->max_nk, h->max_nu, sweep_variant(h), ng, R, nt, h->nsplit,
                                 h->nports, vals_of<T>(h), h->d_bsplit.as<T>(), h->d_twin.as<int32_t>(),
                                 invz_of<T>(h), h->d_o[cur].as<T>(), h->d_o[1 - cur].as<T>(), h->d_xloc.as<T>(),
                                 nullptr, last ? vtm::kSweepWriteX : 0, h->stream);
    };
    // Batches of kGraphBatch sweeps (even, so the wave buffer returns to its start) are captured once
    // per starting buffer and replayed; the remaining sweeps, including the last, are launched directly.
    constexpr int64_t kGraphBatch = 8;
    const int64_t nrep = h->opt.graph_mode == 0 ? (count - 1) / kGraphBatch : 0;
    if (nrep > 0) {
        auto &g = h->graphs[h->cur];
        const void *ptrs[8] = {schur ? (const void *)green_of<T>(h) : (const void *)vals_of<T>(h),
                               schur ? h->d_cport.p : h->d_bsplit.p, h->d_twin.p, invz_of<T>(h), h->d_o[0].p,
                               h->d_o[1].p, h->d_xloc.p, h->mask_on ? h->d_active.p : nullptr};
        bool same = g.exec && g.count == kGraphBatch && g.R == R && g.ng == ng && g.threads == nt &&
                    g.variant == sweep_variant(h) + (schur ? 10 : 0) && g.nlaunch == nsub_launch(h);
        for (int i = 0; i < 8 && same; ++i) same = g.ptrs[i] == ptrs[i];
        if (!same) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            g = vtm_ctx::SweepGraph();
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
            int c = h->cur;
            for (int64_t i = 0; i < kGraphBatch; ++i) {
                launch(c, false);
                c ^= 1;
            }
            HIP_TRY(hipStreamEndCapture(h->stream, &graph));
            hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIP_TRY(e);
            g.count = kGraphBatch;
            g.R = R;
            g.ng = ng;
            g.threads = nt;
            g.variant = sweep_variant(h) + (schur ? 10 : 0);
            for (int i = 0; i < 8; ++i) g.ptrs[i] = ptrs[i];
            g.nlaunch = nsub_launch(h);
        }
        for (int64_t r = 0; r < nrep; ++r) HIP_TRY(hipGraphLaunch(g.exec, h->stream));
    }
    for (int64_t i = nrep * kGraphBatch; i < count; ++i) {
        launch(h->cur, i == count - 1);
        h->cur ^= 1;
    }
    h->waves_zero = false;
    return VTM_OK;
}

// Substitution solve with the incoming waves of the last sweep (or zero waves), local solutions to xloc;
// the waves are not advanced.  write_y also keeps y = L^{-1} (right side) in yb.
template <typename T>
void local_solve(vtm_ctx *h, bool zero_waves, bool write_y = false) {
    const int32_t R = h->wave_R, ng = (h->wave_nrhs + R - 1) / R;
    vtm::launch_sweep<T>(dev_sym(h), dev_sub(h), nsub_launch(h), h->max_nk, h->max_nu, sweep_variant(h), ng, R,
                         sweep_threads(h), h->nsplit, h->nports, vals_of<T>(h), h->d_bsplit.as<T>(),
                         h->d_twin.as<int32_t>(), invz_of<T>(h), h->d_o[h->cur ^ 1].as<T>(), h->d_o[h->cur].as<T>(),
                         h->d_xloc.as<T>(), write_y ? h->d_yb.as<T>() : nullptr,
                         vtm::kSweepWriteX | vtm::kSweepNoWaves | (zero_waves ? vtm::kSweepZeroWaves : 0) |
                             (write_y ? vtm::kSweepWriteY : 0),
                         h->stream);
}

// Y blocks of the port Green's columns in the sweep precision (FP64 workspace or its FP32 copy).
template <typename T>
const T *yblocks_of(vtm_ctx *h);
template <>
const double *yblocks_of<double>(vtm_ctx *h) { return h->d_gws.as<double>(); }
template <>
const float *yblocks_of<float>(vtm_ctx *h) { return h->d_gws32.as<float>(); }

// Local solutions of a convergence test (incoming waves of the last sweep): from the stored Y blocks
// and y_b when the set-up kept them, else by substitution.
template <typename T>
vtm_status test_solve(vtm_ctx *h) {
    const int32_t R = h->wave_R, ng = (h->wave_nrhs + R - 1) / R;
    if (h->have_y && h->yb_ok && vtm::prepare_ysolve<T>(h->max_nk, h->max_p, R) == hipSuccess) {
        vtm::launch_ysolve<T>(dev_sym(h), dev_sub(h), dev_green(h, true), yblocks_of<T>(h), nsub_launch(h), h->max_nk,
                              h->max_p, ng, R, sweep_threads(h), h->nsplit, h->nports, vals_of<T>(h), h->d_yb.as<T>(),
                              h->d_twin.as<int32_t>(), invz_of<T>(h), h->d_o[h->cur ^ 1].as<T>(), h->d_xloc.as<T>(),
                              h->stream);
        return VTM_OK;
    }
    (void)hipGetLastError();
    local_solve<T>(h, false);
    return VTM_OK;
}

// After a new source split: c = K^{-1} b~ at the port vertices (port-reduced sweeps only), and
// y_b = L^{-1} b~ for the tests when the Y blocks are kept.
template <typename T>
vtm_status port_constants(vtm_ctx *h) {
    if (!use_schur(h)) return VTM_OK;
    const int32_t R = h->wave_R, ng = (h->wave_nrhs + R - 1) / R;
    HIP_TRY(vtm::prepare_sweep<T>(h->max_nk, h->max_nu, sweep_variant(h), R));
    HIP_TRY(ensure(h->d_cport, sizeof(T) * ((size_t)ng * h->npg * R + 1)));
    h->yb_ok = false;
    if (h->have_y) {
        HIP_TRY(ensure(h->d_yb, sizeof(T) * ((size_t)ng * h->nsplit * R + 1)));
        h->yb_ok = true;
    }
    local_solve<T>(h, true, h->yb_ok);
    vtm::launch_gather_ports<T>(dev_sub(h), nsub_launch(h), ng, h->nsplit, h->npg, R, h->d_xloc.as<T>(),
                                h->d_cport.as<T>(), h->stream);
    return VTM_OK;
}

template <typename T>
vtm_status alloc_solve(vtm_ctx *h, int32_t nrhs) {
    const int32_t R = h->wave_R, ng = (nrhs + R - 1) / R;
    const int64_t n = h->P.n, S = vtm::vec_stride(nrhs);
    HIP_TRY(ensure(h->d_bsplit, sizeof(T) * (size_t)ng * h->nsplit * R));
    HIP_TRY(ensure(h->d_xloc, sizeof(T) * (size_t)ng * h->nsplit * R));
    HIP_TRY(ensure(h->d_x, sizeof(double) * (size_t)n * S));
    HIP_TRY(ensure(h->d_xt, sizeof(double) * (size_t)n * S));
    HIP_TRY(ensure(h->d_r, sizeof(double) * (size_t)n * S));
    HIP_TRY(ensure(h->d_rt, sizeof(double) * (size_t)n * S));
    HIP_TRY(ensure(h->d_part, sizeof(double) * 2 * (size_t)h->nchunks * nrhs));
    HIP_TRY(ensure(h->d_relres, sizeof(double) * ((size_t)h->P.nsys * nrhs + 1)));
    return VTM_OK;
}

// FP64 residual of x against the staged b; optional store of r; relres to host.
vtm_status residual(vtm_ctx *h, int32_t nrhs, const double *x, double *r, std::vector<double> &rel) {
    vtm::DevCsr A{h->d_rp.as<int64_t>(), h->d_ci.as<int32_t>(), h->d_v.as<double>()};
    const int64_t n = h->P.n;
    vtm::launch_residual(A, n, nrhs, vtm::vec_stride(nrhs), h->d_b.as<double>(), x, r, h->d_chunkrow.as<int64_t>(),
                         h->d_chunksys.as<int32_t>(), h->mask_on ? h->d_active.as<int32_t>() : nullptr, h->nchunks, h->d_syschunk.as<int32_t>(), h->P.nsys,
                         h->d_part.as<double>(), h->abort_pending ? h->d_abort.as<int32_t>() : nullptr,
                         h->d_relres.as<double>(), h->stream);
    rel.resize((size_t)h->P.nsys * nrhs);
    // The norms (and the persistent sweeps' abort flag after them) go to pinned memory and the host
    // polls the copy's completion: a blocking synchronisation would add its wake-up latency to every test.
    const size_t cnt = rel.size() + 1;
    if (h->relres_cap < cnt) {
        if (h->relres_host) HIP_TRY(hipHostFree(h->relres_host));
        h->relres_host = nullptr;
        h->relres_cap = 0;
        HIP_TRY(hipHostMalloc((void **)&h->relres_host, sizeof(double) * cnt, hipHostMallocDefault));
        h->relres_cap = cnt;
    }
    if (!h->ev_test) HIP_TRY(hipEventCreateWithFlags(&h->ev_test, hipEventDisableTiming));
    HIP_TRY(hipMemcpyAsync(h->relres_host, h->d_relres.p, sizeof(double) * cnt, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipEventRecord(h->ev_test, h->stream));
    hipError_t q;
    while ((q = hipEventQuery(h->ev_test)) == hipErrorNotReady) {
    }
    HIP_TRY(q);
    std::copy(h->relres_host, h->relres_host + rel.size(), rel.begin());
    return check_abort(h, h->relres_host[rel.size()] != 0.0 ? 1 : 0);
}

// Cost of one convergence test in sweeps, from a fixed model: algorithmic bytes over a nominal
// stream bandwidth, plus launch latencies (a persistent sweep is bound by the latency of its wave
// exchange, a launched one by the launch).  The test placement uses it instead of measured timings,
// so the placement -- and every reported sweep count -- depends on the iteration alone.
double test_cost_sweeps(vtm_ctx *h, int32_t nrhs, bool schur, bool persistent) {
    constexpr double kBw = 5e12, kSweepPersist = 4e-6, kSweepLaunch = 12e-6, kTestLatency = 60e-6;
    const double s = (double)h->tsize(), r = (double)nrhs;
    const double sweep_bytes = schur ? s * ((persistent ? 0.0 : (double)h->total_g) + (double)h->npg * r +
                                            2.0 * (double)h->nports * r)
                                     : s * ((double)h->total_lower + (double)h->nsplit * r + 2.0 * (double)h->nports * r);
    const double t_sweep = std::max(sweep_bytes / kBw, persistent ? kSweepPersist : kSweepLaunch);
    const double nnz = (double)h->A.rp[h->P.n], n = (double)h->P.n;
    double test_bytes = r * (12.0 * nnz + 24.0 * n) + r * (double)h->nsplit * (s + 8.0);  // residual, merge
    test_bytes += schur ? s * ((double)h->gws_total + 2.0 * (double)h->nsplit * r)       // Y blocks, y_b, x
                        : s * ((double)h->total_lower + 2.0 * (double)h->nsplit * r);    // substitution
    return (test_bytes / kBw + kTestLatency) / t_sweep;
}

// Per-system done mask of a solve over several independent systems: all systems active.
vtm_status mask_begin(vtm_ctx *h) {
    h->mask_on = false;
    const int32_t nsys = h->P.nsys;
    if (nsys <= 1) return VTM_OK;
    if (h->active_cap < (size_t)nsys) {
        if (h->active_host) HIP_TRY(hipHostFree(h->active_host));
        h->active_host = nullptr;
        h->active_cap = 0;
        HIP_TRY(hipHostMalloc((void **)&h->active_host, sizeof(int32_t) * nsys, hipHostMallocDefault));
        h->active_cap = nsys;
    }
    HIP_TRY(ensure(h->d_active, sizeof(int32_t) * nsys));
    std::fill(h->active_host, h->active_host + nsys, 1);
    HIP_TRY(hipMemcpyAsync(h->d_active.p, h->active_host, sizeof(int32_t) * nsys, hipMemcpyHostToDevice, h->stream));
    h->mask_on = true;
    h->list_on = false;
    return VTM_OK;
}

// After systems have converged: the launch list = the subgraphs of the systems still sweeping, in
// launch order (largest G_k first).  The host list stays unchanged until the next rebuild, which
// comes after a synchronisation (a test), so the asynchronous copy from it is safe.
vtm_status mask_relist(vtm_ctx *h) {
    h->h_sublist.clear();
    for (const int32_t k : h->h_gorder)
        if (h->active_host[h->P.sub_sys[k]]) h->h_sublist.push_back(k);
    // sized for every subgraph, so that its address (captured in sweep graphs) never changes
    HIP_TRY(ensure(h->d_sublist, sizeof(int32_t) * std::max<size_t>(h->P.nsub, 1)));
    if (h->h_sublist.empty()) return VTM_OK;  // every system has converged: no further launch
    if (!h->h_sublist.empty())
        HIP_TRY(hipMemcpyAsync(h->d_sublist.p, h->h_sublist.data(), sizeof(int32_t) * h->h_sublist.size(),
                               hipMemcpyHostToDevice, h->stream));
    h->list_on = true;
    return VTM_OK;
}

// Restart the refinement of the systems in sys on their new residuals (rows of r): source split and
// zero waves on their subgraphs, then their port constants, while the other systems go on with their
// current inner solves.  Like the launch list, the host list stays unchanged until the next test's
// synchronisation, so the asynchronous copy from it is safe.
template <typename T>
vtm_status restart_systems(vtm_ctx *h, const std::vector<int32_t> &sys, const double *r, int32_t nrhs) {
    std::vector<char> on(h->P.nsys, 0);
    for (const int32_t s : sys) on[s] = 1;
    h->h_rlist.clear();
    for (const int32_t k : h->h_gorder)
        if (on[h->P.sub_sys[k]]) h->h_rlist.push_back(k);
    if (h->h_rlist.empty()) return VTM_OK;
    HIP_TRY(ensure(h->d_rlist, sizeof(int32_t) * std::max<size_t>(h->P.nsub, 1)));
    HIP_TRY(hipMemcpyAsync(h->d_rlist.p, h->h_rlist.data(), sizeof(int32_t) * h->h_rlist.size(),
                           hipMemcpyHostToDevice, h->stream));
    h->rl_on = true;
    struct ListOff {
        vtm_ctx *h;
        ~ListOff() { h->rl_on = false; }
    } list_off{h};
    vtm::launch_restart<T>(dev_sub(h), dev_maps(h), h->P.nsub, (int32_t)h->h_rlist.size(), h->nsplit, h->nports, r,
                           nrhs, vtm::vec_stride(nrhs), h->wave_R, h->d_bsplit.as<T>(), h->d_o[h->cur].as<T>(),
                           h->stream);
    return port_constants<T>(h);
}

// The VTM solve (Table 1 steps 3-6) on the right sides staged in d_b (waves and buffers ready).
// it[c * nsys + s]: first passing sweep; rel: the relative residuals of the returned x, *xfinal.
//
// Every independent system runs its own course: it stops sweeping once all its right sides pass (done
// mask), and in FP32_IR its inner solve restarts on its new residual once the residual has fallen by
// a factor eta since its last restart, or stalls (then the system stops if it has not improved).
template <typename T>
vtm_status solve_core(vtm_ctx *h, int32_t nrhs, double tol, std::vector<int32_t> &it, std::vector<double> &rel_x,
                      const double **xfinal) {
    vtm_status rc;
    h->stats.persistent = 0;
    h->persist_launches = 0;
    const int64_t n = h->P.n;
    const int32_t nsys = h->P.nsys, R = h->wave_R, ng = (nrhs + R - 1) / R, S = vtm::vec_stride(nrhs);
    const vtm::DevMaps M = dev_maps(h);
    // Test placement: a fixed cadence, or (check_every == 0) from the contraction rate each system
    // showed between its last tests.  Its next event (converged, or refinement step due) is predicted
    // that many sweeps ahead, plus a margin of half the prediction but at most the modelled cost of a
    // test (the rate measured early is faster than the asymptotic one, and a test that falls short
    // costs another).  The next test comes at the earliest event, or at a later one while the sweeps
    // the systems with earlier events would spend waiting cost less than one more test; between 5 and
    // 200 sweeps.  A restart keeps the system's rate (the operator is the same).
    const bool adaptive = h->opt.check_every <= 0;
    int64_t cadence = adaptive ? 10 : h->opt.check_every;
    const int64_t maxsw = h->opt.max_sweeps > 0 ? h->opt.max_sweeps : 100000;
    const bool refine = sizeof(T) == 4;
    const size_t nq = (size_t)nsys * nrhs;
    std::vector<double> rel;
    it.assign(nq, -1);
    std::vector<double> acc_rel(nq, 1.0);     // residuals of the accepted x (x = 0 at the start: r = b)
    std::vector<double> cand_rel(nq, 1e300);  // residuals of the candidate left in xtr (refinement)
    // per system: 0 sweeping, 1 converged, 2 refinement stalled above the tolerance
    std::vector<char> state(nsys, 0);
    struct SysCourse {
        double outer = 1.0;  // worst residual when the current inner solve started
        double prev = 1e300; // worst residual at the previous test of the current inner solve
        double ref = -1.0;   // same, for the rate (not set on the first test after a restart)
        double lr = 0.0;     // last measured log contraction per sweep (< 0 when known)
        int32_t checks = 0;  // tests of the current inner solve
        int32_t steps = 1;   // refinement steps so far
    };
    std::vector<SysCourse> sc(nsys);
    int32_t nactive = nsys;
    Events ev;
    HIP_TRY(ev.create(5));
    const hipEvent_t e0 = ev[0], e1 = ev[1], s0 = ev[2], s1 = ev[3];
    HIP_TRY(hipEventRecord(e0, h->stream));
    if ((rc = mask_begin(h))) return rc;
    struct MaskOff {  // the mask applies to this solve only
        vtm_ctx *h;
        ~MaskOff() { h->mask_on = h->list_on = false; }
    } mask_off{h};
    const int64_t *chunkrow = h->d_chunkrow.as<int64_t>();
    const int32_t *chunksys = h->d_chunksys.as<int32_t>();
    double sweep_ms = 0.0, sweep_bytes = 0.0;
    int64_t sweeps = 0;
    int32_t checks = 0;
    bool diverged = false;
    double first = -1.0;
    // x = 0, r = b for the refinement; the FP64 path solves b directly
    double *xcur = h->d_x.as<double>(), *xtr = h->d_xt.as<double>();
    double *rcur = h->d_r.as<double>(), *rtr = h->d_rt.as<double>();
    // Row moves of a test, per system (1: x from xtr to xcur; 2: also r from rtr to rcur; 3: x from xcur
    // to xtr), done together by one kernel over the residual chunks (one copy per buffer for a single
    // system).  The pinned flag array is rewritten only after the previous upload has completed.
    std::vector<int32_t> rowflag(nsys, 0);
    bool rowflag_pending = false;  // an upload of the flags may still be in flight
    auto flush_rows = [&]() -> vtm_status {
        bool any = false;
        for (const int32_t f : rowflag) any = any || f != 0;
        if (!any) return VTM_OK;
        if (nsys == 1) {
            const size_t bytes = sizeof(double) * (size_t)n * S;
            const int32_t f = rowflag[0];
            HIP_TRY(hipMemcpyAsync(f == 3 ? xtr : xcur, f == 3 ? xcur : xtr, bytes, hipMemcpyDeviceToDevice, h->stream));
            if (f == 2) HIP_TRY(hipMemcpyAsync(rcur, rtr, bytes, hipMemcpyDeviceToDevice, h->stream));
            rowflag[0] = 0;
            return VTM_OK;
        }
        if (h->rowflag_cap < (size_t)nsys) {
            HIP_TRY(hipStreamSynchronize(h->stream));
            if (h->rowflag_host) HIP_TRY(hipHostFree(h->rowflag_host));
            h->rowflag_host = nullptr;
            h->rowflag_cap = 0;
            HIP_TRY(hipHostMalloc((void **)&h->rowflag_host, sizeof(int32_t) * nsys, hipHostMallocDefault));
            h->rowflag_cap = nsys;
            rowflag_pending = false;
        }
        if (rowflag_pending) HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(ensure(h->d_rowflag, sizeof(int32_t) * nsys));
        std::copy(rowflag.begin(), rowflag.end(), h->rowflag_host);
        HIP_TRY(hipMemcpyAsync(h->d_rowflag.p, h->rowflag_host, sizeof(int32_t) * nsys, hipMemcpyHostToDevice,
                               h->stream));
        rowflag_pending = true;
        vtm::launch_sys_rows(chunkrow, chunksys, h->nchunks, h->d_rowflag.as<int32_t>(), S, xcur, xtr, rcur, rtr,
                             h->stream);
        std::fill(rowflag.begin(), rowflag.end(), 0);
        return VTM_OK;
    };
    HIP_TRY(hipMemsetAsync(xcur, 0, sizeof(double) * n * S, h->stream));
    vtm::launch_split<T>(M, h->nsplit, h->d_b.as<double>(), nrhs, S, R, h->d_bsplit.as<T>(), h->stream);
    if ((rc = zero_waves<T>(h))) return rc;
    if ((rc = port_constants<T>(h))) return rc;
    const bool schur = use_schur(h);
    const double test_sweeps = test_cost_sweeps(h, nrhs, schur, schur && persistent_ok(h, R, ng));
    const double eta = 1e-5;
    constexpr double kMargin = 0.5;
    // algorithmic bytes of one sweep of each system (the weights of the test placement)
    std::vector<double> wsys(nsys);
    for (int32_t y = 0; y < nsys; ++y)
        wsys[y] = schur ? h->sys_g[y] + nrhs * (h->sys_pg[y] + 2.0 * h->sys_ports[y])
                        : h->sys_lower[y] + nrhs * (h->sys_split[y] + 2.0 * h->sys_ports[y]);
    std::vector<int32_t> restart;
    std::vector<std::pair<double, double>> events;
    while (nactive > 0 && sweeps < maxsw) {
        const int64_t cnt = std::min(cadence, maxsw - sweeps);
        HIP_TRY(hipEventRecord(s0, h->stream));
        const int64_t launches_before = h->persist_launches;
        if ((rc = run_sweeps_dev<T>(h, cnt))) return rc;
        HIP_TRY(hipEventRecord(s1, h->stream));
        {  // algorithmic bytes of these sweeps over the systems still sweeping
            const double ts = (double)sizeof(T), r = (double)nrhs;
            const double g_reads = h->persist_launches > launches_before
                                       ? (double)(h->persist_launches - launches_before) : (double)cnt;
            for (int32_t y = 0; y < nsys; ++y) {
                if (state[y]) continue;
                sweep_bytes += schur ? ts * (h->sys_g[y] * g_reads + (double)cnt * r * (h->sys_pg[y] + 2.0 * h->sys_ports[y]))
                                     : ts * (double)cnt * (h->sys_lower[y] + r * (h->sys_split[y] + 2.0 * h->sys_ports[y]));
            }
        }
        sweeps += cnt;
        ++checks;
        if (schur && (rc = test_solve<T>(h))) return rc;  // interior potentials of the last sweep
        // merged potentials (plus the refined x in FP32_IR), FP64 residual
        vtm::launch_merge<T>(M, h->nsplit, nrhs, S, R, h->d_xloc.as<T>(), refine ? xcur : nullptr, xtr, chunkrow,
                             chunksys, h->nchunks, h->mask_on ? h->d_active.as<int32_t>() : nullptr, h->stream);
        if ((rc = residual(h, nrhs, xtr, refine ? rtr : nullptr, rel))) return rc;
        rowflag_pending = false;  // the residual's copy to the host has completed: so have earlier uploads
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, s0, s1));
        sweep_ms += ms;
        // the residuals of systems that have stopped are stale: only the sweeping ones count
        double worst = 0.0;
        for (int32_t s = 0; s < nsys; ++s) {
            if (state[s]) continue;
            for (int32_t c = 0; c < nrhs; ++c) {
                const size_t q = (size_t)c * nsys + s;
                if (!std::isfinite(rel[q])) diverged = true;
                if (it[q] < 0 && rel[q] <= tol) it[q] = (int32_t)sweeps;
                worst = std::max(worst, rel[q]);
            }
        }
        if (first < 0) first = worst;
        if (worst > 1e3 * std::max(first, 1.0)) diverged = true;
        if (diverged) {
            cand_rel = rel;
            break;
        }
        restart.clear();
        bool changed = false;  // the done mask changed
        for (int32_t s = 0; s < nsys; ++s) {
            if (state[s]) continue;
            double ws = 0.0;
            bool ok = true;
            for (int32_t c = 0; c < nrhs; ++c) {
                ws = std::max(ws, rel[(size_t)c * nsys + s]);
                ok = ok && rel[(size_t)c * nsys + s] <= tol;
            }
            SysCourse &y = sc[s];
            if (y.ref > 0.0 && ws < y.ref) y.lr = std::log(ws / y.ref) / (double)cnt;
            y.ref = ws;
            ++y.checks;
            if (ok) {  // converged: the candidate is the result, and both x buffers hold it from now on
                state[s] = 1;
                --nactive;
                rowflag[s] = 1;
                for (int32_t c = 0; c < nrhs; ++c) acc_rel[(size_t)c * nsys + s] = rel[(size_t)c * nsys + s];
                changed = true;
                continue;
            }
            if (!refine) continue;
            const bool gained = ws <= 3.0 * eta * y.outer;
            const bool stalled = y.checks >= 2 && ws > 0.995 * y.prev;
            y.prev = ws;
            for (int32_t c = 0; c < nrhs; ++c) cand_rel[(size_t)c * nsys + s] = rel[(size_t)c * nsys + s];
            if ((gained || stalled) && ws < y.outer) {  // accept the candidate, restart on its residual
                restart.push_back(s);
                for (int32_t c = 0; c < nrhs; ++c) {
                    acc_rel[(size_t)c * nsys + s] = rel[(size_t)c * nsys + s];
                    cand_rel[(size_t)c * nsys + s] = 1e300;  // xtr is about to hold an older x
                }
                y.outer = ws;
                y.prev = 1e300;
                y.ref = -1.0;
                y.checks = 0;
                ++y.steps;
            } else if (stalled) {  // no further progress: keep the accepted x (the better one) in both buffers
                state[s] = 2;
                --nactive;
                rowflag[s] = 3;
                changed = true;
            }
        }
        if (h->mask_on && changed) {
            for (int32_t s = 0; s < nsys; ++s) h->active_host[s] = state[s] == 0;
            HIP_TRY(hipMemcpyAsync(h->d_active.p, h->active_host, sizeof(int32_t) * nsys, hipMemcpyHostToDevice,
                                   h->stream));
            if ((rc = mask_relist(h))) return rc;
        }
        // the row moves go before any swap of the buffers; a partial restart moves its systems' x and r
        const bool swap_restart = refine && !restart.empty() && (int32_t)restart.size() == nactive;
        if (refine && !swap_restart)
            for (const int32_t s : restart) rowflag[s] = 2;
        if ((rc = flush_rows())) return rc;
        if (!refine) {
            std::swap(xcur, xtr);
            for (int32_t s = 0; s < nsys; ++s)
                if (!state[s])
                    for (int32_t c = 0; c < nrhs; ++c) acc_rel[(size_t)c * nsys + s] = rel[(size_t)c * nsys + s];
        } else if (!restart.empty()) {
            if (swap_restart) {
                // every system still sweeping restarts (the stopped ones hold the same rows in both buffers)
                std::swap(xcur, xtr);
                std::swap(rcur, rtr);
                vtm::launch_split<T>(M, h->nsplit, rcur, nrhs, S, R, h->d_bsplit.as<T>(), h->stream);
                if ((rc = zero_waves<T>(h))) return rc;
                if ((rc = port_constants<T>(h))) return rc;
            } else {
                if ((rc = restart_systems<T>(h, restart, rcur, nrhs))) return rc;
            }
        }
        if (h->trace) {
            std::fprintf(stderr, "vtm test %d: sweeps %lld, sweeping %d, restarts %zu |", checks, (long long)sweeps,
                         nactive, restart.size());
            for (int32_t s = 0; s < nsys; ++s) {
                double ws = 0.0;
                for (int32_t c = 0; c < nrhs; ++c) ws = std::max(ws, rel[(size_t)c * nsys + s]);
                std::fprintf(stderr, " %c%.1e", "s+x"[state[s]], ws);
            }
            std::fprintf(stderr, "\n");
        }
        if (adaptive && nactive > 0) {
            events.clear();
            double wtot = 0.0;
            for (int32_t s = 0; s < nsys; ++s) {
                if (state[s]) continue;
                const SysCourse &y = sc[s];
                const double target = refine ? std::max(tol, eta * y.outer) : tol;
                const double now = y.ref > 0.0 ? y.ref : y.outer;
                double t = y.ref > 0.0 ? 2.0 * (double)cnt : 10.0;  // rate not known yet
                if (y.lr < 0.0) {
                    const double need = std::log(target / now) / y.lr;
                    t = need > 0.0 ? std::ceil(need + std::min(kMargin * need, test_sweeps)) : 5.0;
                }
                events.emplace_back(t, wsys[s]);
                wtot += wsys[s];
            }
            std::sort(events.begin(), events.end());
            double t_next = events[0].first, w_past = 0.0, waiting = 0.0;
            for (size_t i = 1; i < events.size(); ++i) {
                w_past += events[i - 1].second;
                waiting += w_past * (events[i].first - events[i - 1].first);
                if (waiting > test_sweeps * wtot) break;
                t_next = events[i].first;
            }
            cadence = std::max<int64_t>(5, std::min<int64_t>(200, (int64_t)t_next));
        }
    }
    // refinement stopped by max_sweeps: per system, the better of the accepted x and the last candidate
    if (refine && !diverged)
        for (int32_t s = 0; s < nsys; ++s) {
            if (state[s]) continue;
            double cw = 0.0;
            for (int32_t c = 0; c < nrhs; ++c) cw = std::max(cw, cand_rel[(size_t)c * nsys + s]);
            if (cw < sc[s].outer) {
                rowflag[s] = 1;
                for (int32_t c = 0; c < nrhs; ++c) acc_rel[(size_t)c * nsys + s] = cand_rel[(size_t)c * nsys + s];
            }
        }
    if ((rc = flush_rows())) return rc;
    if (diverged) acc_rel = cand_rel;
    bool done = !diverged;
    for (int32_t s = 0; s < nsys; ++s) done = done && state[s] == 1;
    int32_t outer = 1;
    for (int32_t s = 0; s < nsys; ++s) outer = std::max(outer, sc[s].steps);
    HIP_TRY(hipEventRecord(e1, h->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float total = 0.f;
    HIP_TRY(hipEventElapsedTime(&total, e0, e1));
    h->stats.sweeps = sweeps;
    h->stats.outer_steps = outer;
    h->stats.checks = checks;
    h->stats.solve_ms = total;
    h->stats.sweep_ms = sweep_ms;
    h->stats.sweep_bytes = sweep_bytes;
    if (schur) {
        // G_k is read once per launch: every sweep in per-sweep launches, once per batch in persistent ones
        const double g_reads = h->stats.persistent ? (double)h->persist_launches / (double)std::max<int64_t>(1, sweeps) : 1.0;
        h->stats.bytes_per_sweep =
            (double)sizeof(T) * ((double)h->total_g * g_reads + (double)h->npg * nrhs + 2.0 * (double)h->nports * nrhs);
        h->stats.flops_per_sweep = 2.0 * nrhs * h->total_pp;
    } else {
        h->stats.bytes_per_sweep =
            (double)sizeof(T) * ((double)h->total_lower + (double)h->nsplit * nrhs + 2.0 * (double)h->nports * nrhs);
        h->stats.flops_per_sweep = 4.0 * nrhs * (double)h->total_lower;
    }
    h->stats.sweep_mode = schur ? 2 : 1;
    rel_x = acc_rel;
    *xfinal = xcur;
    if (diverged) return fail(VTM_ERR_DIVERGED, "VTM diverged (non-finite or growing residual)");
    if (!done) return fail(VTM_ERR_NOT_CONVERGED, "tolerance not reached within max_sweeps");
    return VTM_OK;
}

template <typename T>
vtm_status solve_impl(vtm_ctx *h, const double *b, int32_t nrhs, int64_t ldb, double tol, double *x, int64_t ldx,
                      int32_t *iters, double *relres) {
    vtm_status rc;
    if ((rc = ensure_waves<T>(h, nrhs))) return rc;
    if ((rc = alloc_solve<T>(h, nrhs))) return rc;
    if ((rc = stage_b(h, b, nrhs, ldb))) return rc;
    std::vector<int32_t> it;
    std::vector<double> rel;
    const double *xf = nullptr;
    const vtm_status st = solve_core<T>(h, nrhs, tol, it, rel, &xf);
    if (st != VTM_OK && st != VTM_ERR_NOT_CONVERGED && st != VTM_ERR_DIVERGED) return st;
    const std::string msg = vtm::last_error_ref();
    if ((rc = write_x(h, xf, x, nrhs, ldx))) return rc;
    if (iters) std::copy(it.begin(), it.end(), iters);
    if (relres) std::copy(rel.begin(), rel.end(), relres);
    if (st != VTM_OK) vtm::last_error_ref() = msg;
    return st;
}

template <typename T>
vtm_status run_impl(vtm_ctx *h, const double *b, int32_t nrhs, int64_t ldb, int64_t nsweeps, double *x, int64_t ldx) {
    vtm_status rc;
    h->stats.persistent = 0;
    h->persist_launches = 0;
    if ((rc = ensure_waves<T>(h, nrhs))) return rc;
    if ((rc = alloc_solve<T>(h, nrhs))) return rc;
    if ((rc = stage_b(h, b, nrhs, ldb))) return rc;
    const int64_t n = h->P.n;
    const vtm::DevMaps M = dev_maps(h);
    const int32_t S = vtm::vec_stride(nrhs);
    vtm::launch_split<T>(M, h->nsplit, h->d_b.as<double>(), nrhs, S, h->wave_R, h->d_bsplit.as<T>(), h->stream);
    h->stats.sweep_mode = use_schur(h) ? 2 : 1;
    if (nsweeps > 0) {
        if ((rc = port_constants<T>(h))) return rc;
        if ((rc = run_sweeps_dev<T>(h, nsweeps))) return rc;
        if (use_schur(h)) local_solve<T>(h, false);
        vtm::launch_merge<T>(M, h->nsplit, nrhs, S, h->wave_R, h->d_xloc.as<T>(), nullptr, h->d_x.as<double>(),
                             h->d_chunkrow.as<int64_t>(), h->d_chunksys.as<int32_t>(), h->nchunks, nullptr, h->stream);
    } else {
        HIP_TRY(hipMemsetAsync(h->d_x.p, 0, sizeof(double) * n * S, h->stream));
    }
    return write_x(h, h->d_x.as<double>(), x, nrhs, ldx);
}

template <typename T>
vtm_status waves_io(vtm_ctx *h, double *a_out, const double *a_in, int32_t nrhs) {
    vtm_status rc;
    if ((rc = ensure_waves<T>(h, nrhs))) return rc;
    const int32_t R = h->wave_R, ng = (nrhs + R - 1) / R;
    const int64_t np = h->nports;
    std::vector<T> o((size_t)ng * np * R);
    const std::vector<int64_t> &tw = h->P.port_twin;
    if (a_out) {
        HIP_TRY(hipMemcpyAsync(o.data(), h->d_o[h->cur].p, sizeof(T) * o.size(), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        for (int32_t c = 0; c < nrhs; ++c) {
            const int32_t g = c / R, cc = c % R;
            for (int64_t p = 0; p < np; ++p) a_out[(int64_t)c * np + p] = (double)o[((size_t)g * np + tw[p]) * R + cc];
        }
    } else {
        std::fill(o.begin(), o.end(), (T)0);
        for (int32_t c = 0; c < nrhs; ++c) {
            const int32_t g = c / R, cc = c % R;
            for (int64_t p = 0; p < np; ++p) o[((size_t)g * np + tw[p]) * R + cc] = (T)a_in[(int64_t)c * np + p];
        }
        HIP_TRY(hipMemcpyAsync(h->d_o[h->cur].p, o.data(), sizeof(T) * o.size(), hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->waves_zero = false;
    }
    return VTM_OK;
}

void ensure_features(vtm_ctx *h) {
    if (!h->feats_ready) {
        vtm::compute_features(h->A, h->P, h->feats);
        h->feats_ready = true;
    }
}

// Z = exp(clamp(MLP(features), ln 1/4, ln 256)) / a_vv for every VTL, on the device.
vtm_status learned_z(vtm_ctx *h) {
    ensure_features(h);
    const vtm::Partition &P = h->P;
    const int64_t nvtl = (int64_t)P.vtl_v.size();
    if (!h->feats_on_dev) {  // features and diagonals depend on the partition only
        std::vector<double> avv(nvtl);
        for (int64_t l = 0; l < nvtl; ++l) avv[l] = P.adiag[P.vtl_v[l]];
        HIP_TRY(upload(h->d_feat, h->feats, h->stream));
        HIP_TRY(upload(h->d_avvl, avv, h->stream));
        h->feats_on_dev = true;
    }
    HIP_TRY(ensure(h->d_pred, sizeof(float) * (nvtl + 1)));
    HIP_TRY(ensure(h->d_z, sizeof(double) * (nvtl + 1)));
    vtm::launch_mlp_predict(h->d_zparams.as<float>(), h->d_feat.as<float>(), nvtl, h->d_pred.as<float>(), h->stream);
    vtm::launch_z_from_pred(h->d_pred.as<float>(), h->d_avvl.as<double>(), nvtl, std::log(0.25), std::log(256.0),
                            h->d_z.as<double>(), h->stream);
    HIP_TRY(hipGetLastError());
    return VTM_OK;
}

// Impedances set, augmentation, factorisation and (when wanted or forced) the port Green's functions.
vtm_status setup_core(vtm_ctx *h, int32_t z_rule, const std::vector<double> &z, bool force_green,
                      const std::vector<double> *invz_port = nullptr) {
    const vtm::Partition &P = h->P;
    hipStream_t st = h->stream;
    {  // every local solve (zero-wave solves, tests, plain sweeps) keeps a subgraph's vectors in LDS
        const size_t need = vtm::sweep_lds_min(h->tsize(), h->max_nk, h->max_nu);
        if (need > vtm::kMaxLds)
            return fail(VTM_ERR_INVALID, "subgraphs too large: " + std::to_string(h->max_nk) +
                                             " local unknowns need " + std::to_string(need / 1024) +
                                             " KiB of LDS per local solve, more than the CU's " +
                                             std::to_string(vtm::kMaxLds / 1024) + " KiB; use more subgraphs");
    }
    if (z_rule == VTM_Z_LEARNED) {
        vtm_status rc = learned_z(h);
        if (rc) return rc;
    } else {
        HIP_TRY(upload(h->d_z, z, st));
    }
    HIP_TRY(ensure(h->d_invz64, sizeof(double) * (h->nports + 1)));
    HIP_TRY(ensure(h->d_invz32, sizeof(float) * (h->nports + 1)));

    HIP_TRY(ensure(h->d_status, sizeof(int32_t) * (P.nsub + 1)));
    DevBuf &ws = h->d_ws;
    HIP_TRY(ensure(ws, sizeof(double) * (h->total_ws + 1)));
    // port Green's functions for port-reduced sweeps (skipped when forced off or too large)
    const bool want_green = !h->coupled && h->max_p > 0 && h->max_p <= 2048 &&
                            (force_green || (h->opt.sweep_mode != 1 && (h->opt.sweep_mode == 2 ||
                                             (double)h->total_g <= kGreenRatio * (double)h->total_lower)));
    if (want_green && h->plan_state == 0) {
        vtm_status rc = build_green_plan(h);
        if (rc) return rc;
    }
    if (want_green && h->plan_state == 1) {
        const void *before = h->d_gws.p;
        HIP_TRY(ensure(h->d_gws, sizeof(double) * (h->gws_total + 2)));
        if (h->d_gws.p != before) h->gws_clean = false;
    }
    Events ev;
    HIP_TRY(ev.create(2));
    const hipEvent_t e0 = ev[0], e1 = ev[1];
    HIP_TRY(hipEventRecord(e0, st));
    if (invz_port) {  // coupled VTLs: the diagonal of Z_j^{-1} at every port, from the host
        std::vector<float> i32(invz_port->begin(), invz_port->end());
        HIP_TRY(upload(h->d_invz64, *invz_port, st));
        HIP_TRY(upload(h->d_invz32, i32, st));
        HIP_TRY(hipStreamSynchronize(st));
    } else {
        vtm::launch_invz(h->d_z.as<double>(), h->d_portvtl.as<int32_t>(), h->d_invz64.as<double>(),
                         h->d_invz32.as<float>(), h->nports, st);
    }
    const bool fused = want_green && h->plan_state == 1;
    h->have_y = h->have_y32 = h->yb_ok = false;
    if (fused && h->fp32()) {
        HIP_TRY(ensure(h->d_gws32, sizeof(float) * (h->gws_total + 2)));
        h->have_y32 = true;
    }
    // G_k from the stored Y blocks by k_gram (every entry written once) when the plan order is the
    // port-vertex order; otherwise accumulated inside the factorisation into a cleared G
    const bool gram_apart = fused && h->plan_in_order;
    if (want_green) {
        HIP_TRY(ensure(h->d_G64, sizeof(double) * (h->total_g + 256)));
        if (gram_apart)  // only the spare block past the end, which k_gram does not write
            HIP_TRY(hipMemsetAsync(h->d_G64.as<double>() + h->total_g, 0, sizeof(double) * 256, st));
        else
            HIP_TRY(hipMemsetAsync(h->d_G64.p, 0, sizeof(double) * (h->total_g + 256), st));
        // the port fronts start at zero; every factorisation leaves them zero (each supernode clears
        // the front it consumed), so the workspace is cleared only when new
        if (fused && !h->gws_clean) HIP_TRY(hipMemsetAsync(h->d_gws.p, 0, sizeof(double) * (h->gws_total + 2), st));
    }
    // FP32 sweeps take the factor in FP32 straight from the factorisation; the FP64 copy is kept
    // when the sweeps run in FP64 or the Green's functions come from the substitution fallback
    const bool want64 = !h->fp32() || (want_green && !fused);
    if (want64) HIP_TRY(ensure(h->d_vals64, sizeof(double) * (h->total_val + 1)));
    if (h->fp32()) HIP_TRY(ensure(h->d_vals32, sizeof(float) * (h->total_val + 1)));
    vtm::launch_factor(dev_sym(h), dev_sub(h), P.nsub, h->max_front, h->d_aval.as<double>(),
                       h->d_invz64.as<double>(), want64 ? h->d_vals64.as<double>() : nullptr,
                       h->fp32() ? h->d_vals32.as<float>() : nullptr, ws.as<double>(),
                       h->d_status.as<int32_t>(), dev_green(h, fused), h->d_goff.as<int64_t>(),
                       want_green && !gram_apart ? h->d_G64.as<double>() : nullptr, st);
    if (gram_apart)
        vtm::launch_gram(dev_sym(h), dev_sub(h), P.nsub, h->max_p, dev_green(h, true), h->d_goff.as<int64_t>(),
                         h->d_G64.as<double>(), st);
    h->have_green = false;
    if (want_green) {
        if (!fused)
            vtm::launch_green(dev_sym(h), dev_sub(h), P.nsub, h->max_nk, h->max_nu, h->max_p,
                              h->d_vals64.as<double>(), h->d_goff.as<int64_t>(), h->d_G64.as<double>(), st);
        if (h->fp32()) {
            HIP_TRY(ensure(h->d_G32, sizeof(float) * (h->total_g + 256)));
            vtm::launch_to_f32(h->d_G64.as<double>(), h->d_G32.as<float>(), h->total_g + 256, st);
        }
        h->have_green = true;
        h->have_y = fused;
    }
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipGetLastError());
    std::vector<int32_t> status(P.nsub);
    HIP_TRY(hipMemcpyAsync(status.data(), h->d_status.p, sizeof(int32_t) * P.nsub, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (fused) h->gws_clean = true;  // the factorisation ran to its end
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    h->stats.setup_ms = ms;
    for (int32_t k = 0; k < P.nsub; ++k)
        if (status[k]) {
            h->set_up = false;
            return fail(VTM_ERR_NOT_SPD, "non-positive pivot in subgraph " + std::to_string(k) + " (supernode " +
                                             std::to_string(status[k] - 1) + ")");
        }
    static std::atomic<uint64_t> next_setup_id{1};
    h->set_up = true;
    h->setup_id = next_setup_id++;
    h->wave_nrhs = 0;  // fresh zero waves on the next solve
    h->drop_graphs();
    return VTM_OK;
}

// Input impedance of every port (Definition 7.1) with the other ports terminated by their current Z:
// with g the diagonal entry of G_k = R K_k^{-1} R^T at the port's vertex, removing the port's own
// termination 1/Z_p from K_k gives r = 1 / (1/g - 1/Z_p) (Sherman-Morrison).  Needs G.
vtm_status port_rin(vtm_ctx *h, const std::vector<double> &z, std::vector<double> &r) {
    if (!h->have_green) return fail(VTM_ERR_STATE, "input impedances need the port Green's functions");
    DevBuf gd;
    HIP_TRY(ensure(gd, sizeof(double) * (h->npg + 1)));
    vtm::launch_gdiag(dev_sub(h), h->P.nsub, h->d_goff.as<int64_t>(), h->d_G64.as<double>(), gd.as<double>(), h->stream);
    std::vector<double> g(h->npg);
    HIP_TRY(hipMemcpyAsync(g.data(), gd.p, sizeof(double) * h->npg, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    gd.release();
    r.assign(h->nports, 0.0);
    for (int32_t q = 0; q < h->npg; ++q)
        for (int32_t j = 0; j < h->h_pgcnt[q]; ++j) {
            const int64_t p = h->h_pgbeg[q] + j;
            const double d = 1.0 / g[q] - 1.0 / z[h->P.port_vtl[p]];
            r[p] = d > 1e-14 / g[q] ? 1.0 / d : std::numeric_limits<double>::infinity();
        }
    return VTM_OK;
}

// Impedance matching (Section 7.1): starting from the diagonal rule, kMatchIters times set every VTL's
// Z to the geometric mean of its two ports' input impedances (each near "the input impedance of
// either port"), within [1/4, 4096] / a_vv, and set up again.
constexpr int kMatchIters = 2;

vtm_status matched_setup(vtm_ctx *h) {
    const vtm::Partition &P = h->P;
    const int64_t nvtl = (int64_t)P.vtl_v.size();
    if (h->max_p > 2048) return fail(VTM_ERR_INVALID, "impedance matching needs at most 2048 port vertices per subgraph");
    std::vector<int64_t> ends(2 * nvtl, -1);
    for (int64_t p = 0; p < (int64_t)P.port_vtl.size(); ++p) {
        const int64_t l = P.port_vtl[p];
        ends[2 * l + (ends[2 * l] < 0 ? 0 : 1)] = p;
    }
    std::vector<double> z = P.zdiag, r;
    double total_ms = 0.0;
    for (int it = 0; it < kMatchIters; ++it) {
        vtm_status rc = setup_core(h, VTM_Z_USER, z, true);
        if (rc) return rc;
        total_ms += h->stats.setup_ms;
        if ((rc = port_rin(h, z, r))) return rc;
        for (int64_t l = 0; l < nvtl; ++l) {
            const double a = r[ends[2 * l]], b = r[ends[2 * l + 1]];
            const double m = std::sqrt(a) * std::sqrt(b);
            z[l] = std::min(std::max(std::isfinite(m) ? m : 1e300, 0.25 * P.zdiag[l]), 4096.0 * P.zdiag[l]);
        }
    }
    vtm_status rc = setup_core(h, VTM_Z_USER, z, false);
    h->stats.setup_ms += total_ms;
    return rc;
}


// The EVS pieces back in the partition after a coupled set-up, with their own symbolic analysis.
vtm_status restore_pieces(vtm_ctx *h) {
    if (!h->coupled) return VTM_OK;
    h->P.lrp.swap(h->lrp0);
    h->P.lcol.swap(h->lcol0);
    h->P.lval.swap(h->lval0);
    h->lrp0.clear();
    h->lcol0.clear();
    h->lval0.clear();
    h->coupled = false;
    h->set_up = false;
    std::string err;
    const int leaf = h->opt.leaf_size > 0 ? h->opt.leaf_size : 16;
    int rc = vtm::build_symbolic(h->P, leaf, h->S, err);
    if (rc) return fail(rc, err);
    return upload_partition(h);
}

// Coupled VTLs (Section 7.2, Theorem 7.1).  Z is a symmetric matrix over the VTLs: diagonal z_vtl,
// off-diagonal entries zab[e] at (la[e], lb[e]); coupled VTLs must join the same two subgraphs, so
// that Z is block diagonal over groups of VTLs between one pair of subgraphs and both subgraphs of a
// group use its block, in their own port order, as their Z_j (the twins then see one matrix).  Each
// block is factored Z = L L^T (failure: not SPD) and inverted as L^{-T} L^{-1}.  The local matrix
// of (5.8) gets the block Z_j^{-1} on the group's port vertices: its diagonal through the port
// diagonal, its other entries as added entries of the local pieces (which may widen their sparsity,
// so the symbolic analysis is redone); each sweep adds sum_q (Z_j^{-1})_pq a_q to the right side.
vtm_status coupled_setup(vtm_ctx *h, const double *z_vtl, int64_t ncpl, const int64_t *la, const int64_t *lb,
                         const double *zab) {
    vtm::Partition &P = h->P;
    const int64_t nvtl = (int64_t)P.vtl_v.size(), np = (int64_t)P.port_v.size();
    std::vector<double> z(z_vtl, z_vtl + nvtl);
    for (int64_t l = 0; l < nvtl; ++l)
        if (!(z[l] > 0.0) || !std::isfinite(z[l])) return fail(VTM_ERR_INVALID, "Z must be finite and > 0");
    for (int64_t e = 0; e < ncpl; ++e) {
        if (la[e] < 0 || la[e] >= nvtl || lb[e] < 0 || lb[e] >= nvtl || la[e] == lb[e] || !std::isfinite(zab[e]))
            return fail(VTM_ERR_INVALID, "coupling entry " + std::to_string(e) + " invalid");
        if (P.vtl_k[la[e]] != P.vtl_k[lb[e]] || P.vtl_k2[la[e]] != P.vtl_k2[lb[e]])
            return fail(VTM_ERR_INVALID, "coupled VTLs " + std::to_string(la[e]) + ", " + std::to_string(lb[e]) +
                                             " do not join the same two subgraphs");
    }
    // groups: connected components of the coupling graph (labels = smallest member)
    std::vector<int64_t> lab(nvtl);
    for (int64_t l = 0; l < nvtl; ++l) lab[l] = l;
    auto find = [&](int64_t x) {
        while (lab[x] != x) x = lab[x] = lab[lab[x]];
        return x;
    };
    for (int64_t e = 0; e < ncpl; ++e) {
        const int64_t a = find(la[e]), b = find(lb[e]);
        if (a != b) lab[std::max(a, b)] = std::min(a, b);
    }
    std::vector<std::vector<int64_t>> members(nvtl);
    std::vector<int32_t> slot(nvtl);
    for (int64_t l = 0; l < nvtl; ++l) {
        const int64_t g = find(l);
        slot[l] = (int32_t)members[g].size();
        members[g].push_back(l);
    }
    std::vector<std::vector<double>> Y(nvtl);  // per group root: Z^{-1}, m x m row-major
    {
        std::vector<std::vector<double>> Zg(nvtl);
        for (int64_t g = 0; g < nvtl; ++g) {
            const size_t m = members[g].size();
            if (!m) continue;
            Zg[g].assign(m * m, 0.0);
            for (size_t i = 0; i < m; ++i) Zg[g][i * m + i] = z[members[g][i]];
        }
        for (int64_t e = 0; e < ncpl; ++e) {
            const int64_t g = find(la[e]);
            const size_t m = members[g].size(), i = slot[la[e]], j = slot[lb[e]];
            Zg[g][i * m + j] = zab[e];
            Zg[g][j * m + i] = zab[e];
        }
        for (int64_t g = 0; g < nvtl; ++g) {
            const size_t m = members[g].size();
            if (!m) continue;
            std::vector<double> L(m * m, 0.0), Li(m * m, 0.0);
            for (size_t j = 0; j < m; ++j) {  // column-oriented Cholesky
                double d = Zg[g][j * m + j];
                for (size_t t = 0; t < j; ++t) d -= L[j * m + t] * L[j * m + t];
                if (!(d > 0.0) || !std::isfinite(d))
                    return fail(VTM_ERR_INVALID, "coupled impedance block of VTL " + std::to_string(members[g][0]) +
                                                     " is not positive definite");
                L[j * m + j] = std::sqrt(d);
                for (size_t i = j + 1; i < m; ++i) {
                    double v = Zg[g][i * m + j];
                    for (size_t t = 0; t < j; ++t) v -= L[i * m + t] * L[j * m + t];
                    L[i * m + j] = v / L[j * m + j];
                }
            }
            for (size_t j = 0; j < m; ++j) {  // Li = L^{-1}, lower triangular
                Li[j * m + j] = 1.0 / L[j * m + j];
                for (size_t i = j + 1; i < m; ++i) {
                    double v = 0.0;
                    for (size_t t = j; t < i; ++t) v -= L[i * m + t] * Li[t * m + j];
                    Li[i * m + j] = v / L[i * m + i];
                }
            }
            Y[g].assign(m * m, 0.0);  // Z^{-1} = Li^T Li
            for (size_t i = 0; i < m; ++i)
                for (size_t j = 0; j < m; ++j) {
                    double v = 0.0;
                    for (size_t t = std::max(i, j); t < m; ++t) v += Li[t * m + i] * Li[t * m + j];
                    Y[g][i * m + j] = v;
                }
        }
    }
    // the two ports of every VTL (end 0 in vtl_k, end 1 in vtl_k2) and the subgraph of every port
    std::vector<int64_t> vport(2 * nvtl);
    std::vector<int32_t> sub_of(np);
    for (int32_t k = 0; k < P.nsub; ++k)
        for (int64_t q = P.port_ptr[k]; q < P.port_ptr[k + 1]; ++q) {
            const int64_t l = P.port_vtl[q];
            vport[2 * l + (k == P.vtl_k[l] ? 0 : 1)] = q;
            sub_of[q] = k;
        }
    std::vector<double> invz(np);
    std::vector<int32_t> cptr(np + 1, 0), ctw;
    std::vector<double> cy;
    // additions to the local pieces: (subgraph, local row, local column, value), off-diagonal only
    struct Add {
        int32_t k, i, j;
        double v;
    };
    std::vector<Add> adds;
    for (int64_t q = 0; q < np; ++q) {
        const int64_t l = P.port_vtl[q], g = find(l);
        const int end = vport[2 * l] == q ? 0 : 1;
        const size_t m = members[g].size(), i = slot[l];
        invz[q] = Y[g][i * m + i];
        for (size_t j = 0; j < m; ++j) {
            if (j == i) continue;
            const int64_t qo = vport[2 * members[g][j] + end];
            ctw.push_back((int32_t)P.port_twin[qo]);
            cy.push_back(Y[g][i * m + j]);
            adds.push_back(Add{sub_of[q], P.port_lidx[q], P.port_lidx[qo], Y[g][i * m + j]});
        }
        cptr[q + 1] = (int32_t)ctw.size();
    }
    // the EVS pieces with the added entries (kept aside: vtm_get_partition returns the pieces)
    vtm_status rc = restore_pieces(h);
    if (rc) return rc;
    std::sort(adds.begin(), adds.end(), [](const Add &a, const Add &b) {
        return a.k != b.k ? a.k < b.k : a.i != b.i ? a.i < b.i : a.j < b.j;
    });
    std::vector<int64_t> lrp(P.lrp.size());
    std::vector<int32_t> lcol;
    std::vector<double> lval;
    lcol.reserve(P.lcol.size() + adds.size());
    lval.reserve(P.lcol.size() + adds.size());
    size_t ai = 0;
    lrp[0] = 0;
    for (int32_t k = 0; k < P.nsub; ++k)
        for (int64_t r = P.loc_ptr[k]; r < P.loc_ptr[k + 1]; ++r) {
            const int32_t i = (int32_t)(r - P.loc_ptr[k]);
            int64_t e = P.lrp[r];
            const int64_t e1 = P.lrp[r + 1];
            while (e < e1 || (ai < adds.size() && adds[ai].k == k && adds[ai].i == i)) {
                const bool take_add = ai < adds.size() && adds[ai].k == k && adds[ai].i == i &&
                                      (e >= e1 || adds[ai].j <= P.lcol[e]);
                if (take_add) {
                    const Add &a = adds[ai++];
                    if (e < e1 && a.j == P.lcol[e]) {
                        lcol.push_back(P.lcol[e]);
                        lval.push_back(P.lval[e] + a.v);
                        ++e;
                    } else if (!lcol.empty() && (int64_t)lcol.size() > lrp[r] && lcol.back() == a.j) {
                        lval.back() += a.v;
                    } else {
                        lcol.push_back(a.j);
                        lval.push_back(a.v);
                    }
                } else {
                    lcol.push_back(P.lcol[e]);
                    lval.push_back(P.lval[e]);
                    ++e;
                }
            }
            lrp[r + 1] = (int64_t)lcol.size();
        }
    h->lrp0.swap(P.lrp);
    h->lcol0.swap(P.lcol);
    h->lval0.swap(P.lval);
    P.lrp.swap(lrp);
    P.lcol.swap(lcol);
    P.lval.swap(lval);
    h->coupled = true;
    std::string err;
    const int leaf = h->opt.leaf_size > 0 ? h->opt.leaf_size : 16;
    int r2 = vtm::build_symbolic(P, leaf, h->S, err);
    if (r2) return fail(r2, err);
    if ((rc = upload_partition(h))) return rc;
    std::vector<float> cy32(cy.begin(), cy.end());
    HIP_TRY(upload(h->d_cplptr, cptr, h->stream));
    HIP_TRY(upload(h->d_cpltw, ctw, h->stream));
    HIP_TRY(upload(h->d_cply64, cy, h->stream));
    HIP_TRY(upload(h->d_cply32, cy32, h->stream));
    return setup_core(h, VTM_Z_USER, z, false, &invz);
}

// vtm_batch_solve: the members' systems as one block-diagonal set of independent systems (each
// member's systems stay systems of the batch), in a context of its own that holds copies of their
// partitions, symbolic analyses and impedances and factors them again, all in one launch.
vtm_status build_batch(vtm_ctx *const *hs, int32_t count, vtm_ctx *B) {
    vtm::Csr &A = B->A;
    vtm::Partition &P = B->P;
    vtm::Symbolic &S = B->S;
    A = vtm::Csr();
    P = vtm::Partition();
    S = vtm::Symbolic();
    A.rp.assign(1, 0);
    P.s_ptr.assign(1, 0);
    P.loc_ptr.assign(1, 0);
    P.lrp.assign(1, 0);
    P.port_ptr.assign(1, 0);
    P.sys_ptr.assign(1, 0);
    P.nsys = 0;
    std::vector<double> z;
    for (int32_t i = 0; i < count; ++i) {
        const vtm_ctx *h = hs[i];
        const vtm::Csr &a = h->A;
        const vtm::Partition &p = h->P;
        const int64_t vo = A.n, eo = (int64_t)A.ci.size(), so = (int64_t)P.s_idx.size(), xo = (int64_t)P.loc_vtx.size(),
                      lo = (int64_t)P.lcol.size(), to = (int64_t)P.vtl_v.size(), po = (int64_t)P.port_v.size();
        const int32_t ko = P.nsub, co = (int32_t)S.classes.size(), yo = P.nsys;
        for (int64_t v = 0; v < a.n; ++v) A.rp.push_back(a.rp[v + 1] + eo);
        for (const int32_t c : a.ci) A.ci.push_back((int32_t)(c + vo));
        A.v.insert(A.v.end(), a.v.begin(), a.v.end());
        for (int64_t v = 0; v < p.n; ++v) P.s_ptr.push_back(p.s_ptr[v + 1] + so);
        for (const int32_t k : p.s_idx) P.s_idx.push_back(k + ko);
        for (int32_t k = 0; k < p.nsub; ++k) P.loc_ptr.push_back(p.loc_ptr[k + 1] + xo);
        for (const int64_t v : p.loc_vtx) P.loc_vtx.push_back(v + vo);
        for (size_t e = 1; e < p.lrp.size(); ++e) P.lrp.push_back(p.lrp[e] + lo);
        P.lcol.insert(P.lcol.end(), p.lcol.begin(), p.lcol.end());
        P.lval.insert(P.lval.end(), p.lval.begin(), p.lval.end());
        for (const int64_t v : p.vtl_v) P.vtl_v.push_back(v + vo);
        for (const int32_t k : p.vtl_k) P.vtl_k.push_back(k + ko);
        for (const int32_t k : p.vtl_k2) P.vtl_k2.push_back(k + ko);
        for (int32_t k = 0; k < p.nsub; ++k) P.port_ptr.push_back(p.port_ptr[k + 1] + po);
        for (const int64_t v : p.port_v) P.port_v.push_back(v + vo);
        for (const int64_t t : p.port_twin) P.port_twin.push_back(t + po);
        for (const int64_t l : p.port_vtl) P.port_vtl.push_back(l + to);
        for (const int32_t k : p.port_other) P.port_other.push_back(k + ko);
        P.port_lidx.insert(P.port_lidx.end(), p.port_lidx.begin(), p.port_lidx.end());
        P.adiag.insert(P.adiag.end(), p.adiag.begin(), p.adiag.end());
        P.zdiag.insert(P.zdiag.end(), p.zdiag.begin(), p.zdiag.end());
        for (int32_t y = 0; y < p.nsys; ++y) P.sys_ptr.push_back(p.sys_ptr[y + 1] + vo);
        for (const int32_t y : p.sub_sys) P.sub_sys.push_back(y + yo);
        for (const int32_t c : h->S.sub_class) S.sub_class.push_back(c + co);
        S.classes.insert(S.classes.end(), h->S.classes.begin(), h->S.classes.end());
        A.n += a.n;
        P.n += p.n;
        P.nsub += p.nsub;
        P.nsys += p.nsys;
        std::vector<double> zi(p.vtl_v.size());
        if (!zi.empty())
            HIP_TRY(hipMemcpy(zi.data(), h->d_z.p, sizeof(double) * zi.size(), hipMemcpyDeviceToHost));
        z.insert(z.end(), zi.begin(), zi.end());
    }
    vtm_status rc = upload_partition(B);
    if (rc) return rc;
    B->partitioned = true;
    return setup_core(B, VTM_Z_USER, z, false);
}

template <typename T>
vtm_status batch_impl(vtm_ctx *B, vtm_ctx *const *hs, int32_t count, const double *const *b, int32_t nrhs,
                      const int64_t *ldb, double tol, double *const *x, const int64_t *ldx, int32_t *const *iters,
                      double *const *relres) {
    vtm_status rc;
    if ((rc = ensure_waves<T>(B, nrhs))) return rc;
    if ((rc = alloc_solve<T>(B, nrhs))) return rc;
    const int64_t N = B->P.n, S = vtm::vec_stride(nrhs);
    HIP_TRY(ensure(B->d_b, sizeof(double) * (size_t)N * S));
    int64_t vo = 0;
    for (int32_t i = 0; i < count; ++i) {  // the members' rows one after the other
        const int64_t ni = hs[i]->P.n;
        if ((rc = to_rows(B, b[i], ldb[i], ni, nrhs, B->d_b.as<double>() + vo * S, B->d_rt.as<double>()))) return rc;
        vo += ni;
    }
    std::vector<int32_t> it;
    std::vector<double> rel;
    const double *xf = nullptr;
    const vtm_status st = solve_core<T>(B, nrhs, tol, it, rel, &xf);
    if (st != VTM_OK && st != VTM_ERR_NOT_CONVERGED && st != VTM_ERR_DIVERGED) return st;
    const std::string msg = vtm::last_error_ref();
    vo = 0;
    int32_t yo = 0;
    const int32_t NS = B->P.nsys;
    for (int32_t i = 0; i < count; ++i) {
        const int64_t ni = hs[i]->P.n;
        const int32_t nsi = hs[i]->P.nsys;
        if ((rc = from_rows(B, xf + vo * S, ni, nrhs, x[i], ldx[i], B->d_r.as<double>()))) return rc;
        for (int32_t c = 0; c < nrhs; ++c)
            for (int32_t y = 0; y < nsi; ++y) {
                const size_t q = (size_t)c * NS + yo + y, qi = (size_t)c * nsi + y;
                if (iters && iters[i]) iters[i][qi] = it[q];
                if (relres && relres[i]) relres[i][qi] = rel[q];
            }
        vo += ni;
        yo += nsi;
    }
    HIP_TRY(hipStreamSynchronize(B->stream));
    if ((rc = check_abort(B))) return rc;
    for (int32_t i = 0; i < count; ++i) hs[i]->stats = B->stats;
    if (st != VTM_OK) vtm::last_error_ref() = msg;
    return st;
}

}  // namespace

extern "C" {

const char *vtm_last_error(void) { return vtm::last_error_ref().c_str(); }

vtm_status vtm_create(const vtm_options *options, vtm_handle *out) {
    if (!out) return fail(VTM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    vtm_ctx *h = new (std::nothrow) vtm_ctx();
    if (!h) return fail(VTM_ERR_OOM, "handle allocation failed");
    if (options) h->opt = *options;
    h->trace = std::getenv("VTM_TRACE") != nullptr;
    if (h->opt.precision != VTM_FP64 && h->opt.precision != VTM_FP32_IR) {
        delete h;
        return fail(VTM_ERR_INVALID, "unknown precision");
    }
    if (h->opt.sweep_waves < 0 || h->opt.sweep_waves > 2) {
        delete h;
        return fail(VTM_ERR_INVALID, "sweep_waves must be 0, 1 or 2");
    }
    if (h->opt.spin_limit < 0) {
        delete h;
        return fail(VTM_ERR_INVALID, "spin_limit must be >= 0");
    }
    if (h->opt.device < 0) {  // host-only handle: partition and symbolic analysis, no device work
        *out = h;
        return VTM_OK;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        delete h;
        return fail(VTM_ERR_HIP, "no HIP device available");
    }
    if (h->opt.device < 0 || h->opt.device >= ndev) {
        delete h;
        return fail(VTM_ERR_INVALID, "device ordinal out of range");
    }
    if ((e = hipSetDevice(h->opt.device)) != hipSuccess) {
        delete h;
        return fail(VTM_ERR_HIP, hipGetErrorString(e));
    }
    if (hipDeviceGetAttribute(&h->ncu, hipDeviceAttributeMultiprocessorCount, h->opt.device) != hipSuccess) h->ncu = 0;
    {  // the allocation-free entry points' scratch: its address on this device, looked up once
        double *scr = nullptr;
        if ((e = vtm::noalloc_scratch(h->opt.device, &scr)) != hipSuccess) {
            delete h;
            return fail(VTM_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(e));
        }
    }
    if (h->opt.stream) h->stream = (hipStream_t)h->opt.stream;
    else {
        if ((e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking)) != hipSuccess) {
            delete h;
            return fail(VTM_ERR_HIP, hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    *out = h;
    return VTM_OK;
}

vtm_status vtm_destroy(vtm_handle h) {
    delete h;
    return VTM_OK;
}

vtm_status vtm_evs_partition(vtm_handle h, int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                             const vtm_partition_spec *spec, vtm_partition_info *info) {
    if (!h || !rowptr || !col || !val || !spec || n < 1) return fail(VTM_ERR_INVALID, "null argument or n < 1");
    if (rowptr[0] != 0 || rowptr[n] < n) return fail(VTM_ERR_INVALID, "rowptr invalid");
    if (!h->host_only()) HIP_TRY(hipSetDevice(h->opt.device));
    h->partitioned = h->set_up = false;
    h->feats_ready = h->feats_on_dev = false;
    h->coupled = false;
    h->A.n = n;
    h->A.rp.assign(rowptr, rowptr + n + 1);
    h->A.ci.assign(col, col + rowptr[n]);
    h->A.v.assign(val, val + rowptr[n]);
    std::string err;
    int rc = vtm::build_partition(h->A, *spec, h->P, err);
    if (rc) return fail(rc, err);
    int leaf = h->opt.leaf_size > 0 ? h->opt.leaf_size : 16;
    rc = vtm::build_symbolic(h->P, leaf, h->S, err);
    if (rc) return fail(rc, err);
    if (h->host_only()) host_sizes(h);
    else if ((rc = upload_partition(h))) return rc;
    h->wave_nrhs = 0;
    h->partitioned = true;
    if (info) {
        info->nsub = h->P.nsub;
        info->nclass = (int32_t)h->S.classes.size();
        info->n_split = h->nsplit;
        info->nvtl = (int64_t)h->P.vtl_v.size();
        info->nports = h->nports;
        info->max_local = h->max_nk;
        info->nsys = h->P.nsys;
        info->factor_entries = h->total_lower;
        info->rcb_seed = h->P.rcb_seed;
    }
    return VTM_OK;
}

vtm_status vtm_get_partition(vtm_handle h, int64_t *s_ptr, int32_t *s_idx, int64_t *loc_ptr, int64_t *loc_vtx,
                             int64_t *lrp, int32_t *lcol, double *lval, int64_t *vtl_v, int32_t *vtl_k,
                             int32_t *vtl_k2, int64_t *port_ptr, int64_t *port_v, int32_t *port_other,
                             int64_t *port_twin, double *zdiag) {
    if (!h) return fail(VTM_ERR_INVALID, "null handle");
    if (!h->partitioned) return fail(VTM_ERR_STATE, "no partition");
    const vtm::Partition &P = h->P;
    auto cp = [](auto *dst, const auto &src) {
        if (dst) std::copy(src.begin(), src.end(), dst);
    };
    cp(s_ptr, P.s_ptr); cp(s_idx, P.s_idx); cp(loc_ptr, P.loc_ptr); cp(loc_vtx, P.loc_vtx);
    cp(lrp, h->coupled ? h->lrp0 : P.lrp);  // the EVS pieces, also while a coupled set-up holds the handle
    cp(lcol, h->coupled ? h->lcol0 : P.lcol);
    cp(lval, h->coupled ? h->lval0 : P.lval); cp(vtl_v, P.vtl_v); cp(vtl_k, P.vtl_k); cp(vtl_k2, P.vtl_k2);
    cp(port_ptr, P.port_ptr); cp(port_v, P.port_v); cp(port_other, P.port_other); cp(port_twin, P.port_twin);
    cp(zdiag, P.zdiag);
    return VTM_OK;
}

vtm_status vtm_setup(vtm_handle h, int32_t z_rule, const double *z_vtl) {
    if (!h) return fail(VTM_ERR_INVALID, "null handle");
    if (h->host_only()) return fail(VTM_ERR_STATE, "host-only handle (device < 0) cannot set up");
    if (!h->partitioned) return fail(VTM_ERR_STATE, "vtm_setup before vtm_evs_partition");
    HIP_TRY(hipSetDevice(h->opt.device));
    if (h->coupled) {  // back to the EVS pieces of the partition
        vtm_status rc = restore_pieces(h);
        if (rc) return rc;
    }
    const vtm::Partition &P = h->P;
    const int64_t nvtl = (int64_t)P.vtl_v.size();
    std::vector<double> z;
    if (z_rule == VTM_Z_DIAG) z = P.zdiag;
    else if (z_rule == VTM_Z_USER) {
        if (!z_vtl && nvtl) return fail(VTM_ERR_INVALID, "VTM_Z_USER needs z_vtl");
        z.assign(z_vtl, z_vtl + nvtl);
        for (int64_t l = 0; l < nvtl; ++l)
            if (!(z[l] > 0.0) || !std::isfinite(z[l])) return fail(VTM_ERR_INVALID, "Z must be finite and > 0");
    } else if (z_rule == VTM_Z_LEARNED) {
        if (!h->model_loaded) return fail(VTM_ERR_STATE, "VTM_Z_LEARNED before vtm_zmodel_load");
    } else if (z_rule == VTM_Z_MATCHED) {
        return matched_setup(h);
    } else {
        return fail(VTM_ERR_INVALID, "unknown z_rule");
    }
    return setup_core(h, z_rule, z, false);
}

vtm_status vtm_setup_coupled(vtm_handle h, const double *z_vtl, int64_t ncouple, const int64_t *vtl_a,
                             const int64_t *vtl_b, const double *z_ab) {
    if (!h || (!z_vtl && h->P.vtl_v.size()) || ncouple < 0 || (ncouple > 0 && (!vtl_a || !vtl_b || !z_ab)))
        return fail(VTM_ERR_INVALID, "bad argument");
    if (h->host_only()) return fail(VTM_ERR_STATE, "host-only handle (device < 0) cannot set up");
    if (!h->partitioned) return fail(VTM_ERR_STATE, "vtm_setup_coupled before vtm_evs_partition");
    HIP_TRY(hipSetDevice(h->opt.device));
    h->set_up = false;
    return coupled_setup(h, z_vtl, ncouple, vtl_a, vtl_b, z_ab);
}

vtm_status vtm_input_impedance(vtm_handle h, double *r_port) {
    if (!h || !r_port) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->set_up) return fail(VTM_ERR_STATE, "vtm_input_impedance before vtm_setup");
    HIP_TRY(hipSetDevice(h->opt.device));
    std::vector<double> z(h->P.vtl_v.size()), r;
    HIP_TRY(hipMemcpy(z.data(), h->d_z.p, sizeof(double) * z.size(), hipMemcpyDeviceToHost));
    vtm_status rc = port_rin(h, z, r);
    if (rc) return rc;
    std::copy(r.begin(), r.end(), r_port);
    return VTM_OK;
}

vtm_status vtm_input_impedance_noalloc(vtm_handle h, double *r_port) {
    if (!h || !r_port) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->set_up) return fail(VTM_ERR_STATE, "vtm_input_impedance_noalloc before vtm_setup");
    if (!h->have_green) return fail(VTM_ERR_STATE, "input impedances need the port Green's functions");
    if ((size_t)h->nports > vtm::kNoAllocDoubles)
        return fail(VTM_ERR_INVALID, std::to_string(h->nports) + " ports exceed the scratch of " +
                                         std::to_string(vtm::kNoAllocDoubles) + " values");
    HIP_TRY(hipSetDevice(h->opt.device));
    double *scr = nullptr;
    HIP_TRY(vtm::noalloc_scratch(h->opt.device, &scr));
    if (h->nports == 0) return VTM_OK;
    vtm::launch_rin(dev_sub(h), h->P.nsub, h->d_goff.as<int64_t>(), h->d_G64.as<double>(), h->d_invz64.as<double>(),
                    scr, h->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(r_port, scr, sizeof(double) * (size_t)h->nports,
                           is_device_ptr(r_port) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return VTM_OK;
}

vtm_status vtm_solve(vtm_handle h, const double *b, int32_t nrhs, int64_t ldb, double tol, double *x, int64_t ldx,
                     int32_t *iters, double *relres) {
    if (!h || !b || !x || nrhs < 1) return fail(VTM_ERR_INVALID, "null argument or nrhs < 1");
    if (!h->set_up) return fail(VTM_ERR_STATE, "vtm_solve before vtm_setup");
    if (!(tol > 0.0) || ldb < h->P.n || ldx < h->P.n) return fail(VTM_ERR_INVALID, "tol <= 0 or leading dimension < n");
    HIP_TRY(hipSetDevice(h->opt.device));
    return h->fp32() ? solve_impl<float>(h, b, nrhs, ldb, tol, x, ldx, iters, relres)
                     : solve_impl<double>(h, b, nrhs, ldb, tol, x, ldx, iters, relres);
}

vtm_status vtm_batch_solve(vtm_handle *hs, int32_t count, const double *const *b, int32_t nrhs, const int64_t *ldb,
                           double tol, double *const *x, const int64_t *ldx, int32_t *const *iters,
                           double *const *relres) {
    if (!hs || count < 1 || !b || !x || !ldb || !ldx || nrhs < 1) return fail(VTM_ERR_INVALID, "bad argument");
    if (!(tol > 0.0)) return fail(VTM_ERR_INVALID, "tol <= 0");
    vtm_ctx *h0 = hs[0];
    for (int32_t i = 0; i < count; ++i) {
        vtm_ctx *h = hs[i];
        if (!h || !b[i] || !x[i]) return fail(VTM_ERR_INVALID, "null handle or vector in the batch");
        if (!h->set_up) return fail(VTM_ERR_STATE, "vtm_batch_solve: member " + std::to_string(i) + " is not set up");
        if (h->coupled) return fail(VTM_ERR_INVALID, "vtm_batch_solve: member " + std::to_string(i) + " has coupled VTLs");
        if (h->opt.device != h0->opt.device || h->opt.precision != h0->opt.precision)
            return fail(VTM_ERR_INVALID, "batch members must share the device and the precision");
        if (ldb[i] < h->P.n || ldx[i] < h->P.n) return fail(VTM_ERR_INVALID, "leading dimension < n");
    }
    HIP_TRY(hipSetDevice(h0->opt.device));
    std::vector<uint64_t> key(count);
    for (int32_t i = 0; i < count; ++i) key[i] = hs[i]->setup_id;
    if (!h0->batch || h0->batch_key != key) {
        delete h0->batch;
        h0->batch = nullptr;
        h0->batch_key.clear();
        vtm_ctx *B = new (std::nothrow) vtm_ctx();
        if (!B) return fail(VTM_ERR_OOM, "batch context allocation failed");
        B->opt = h0->opt;
        B->opt.stream = h0->stream;
        B->stream = h0->stream;
        B->own_stream = false;
        vtm_status rc = build_batch(hs, count, B);
        if (rc) {
            delete B;
            return rc;
        }
        h0->batch = B;
        h0->batch_key = key;
    }
    vtm_ctx *B = h0->batch;
    return B->fp32() ? batch_impl<float>(B, hs, count, b, nrhs, ldb, tol, x, ldx, iters, relres)
                     : batch_impl<double>(B, hs, count, b, nrhs, ldb, tol, x, ldx, iters, relres);
}

vtm_status vtm_run_sweeps(vtm_handle h, const double *b, int32_t nrhs, int64_t ldb, int64_t nsweeps, double *x,
                          int64_t ldx) {
    if (!h || !b || !x || nrhs < 1 || nsweeps < 0) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->set_up) return fail(VTM_ERR_STATE, "vtm_run_sweeps before vtm_setup");
    if (ldb < h->P.n || ldx < h->P.n) return fail(VTM_ERR_INVALID, "leading dimension < n");
    HIP_TRY(hipSetDevice(h->opt.device));
    return h->fp32() ? run_impl<float>(h, b, nrhs, ldb, nsweeps, x, ldx)
                     : run_impl<double>(h, b, nrhs, ldb, nsweeps, x, ldx);
}

vtm_status vtm_reset_waves(vtm_handle h) {
    if (!h) return fail(VTM_ERR_INVALID, "null handle");
    if (!h->set_up) return fail(VTM_ERR_STATE, "no setup");
    HIP_TRY(hipSetDevice(h->opt.device));
    if (!h->d_o[0].p) return VTM_OK;
    vtm_status rc = h->fp32() ? zero_waves<float>(h) : zero_waves<double>(h);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return VTM_OK;
}

vtm_status vtm_get_waves(vtm_handle h, double *a, int32_t nrhs) {
    if (!h || !a || nrhs < 1) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->set_up) return fail(VTM_ERR_STATE, "no setup");
    HIP_TRY(hipSetDevice(h->opt.device));
    return h->fp32() ? waves_io<float>(h, a, nullptr, nrhs) : waves_io<double>(h, a, nullptr, nrhs);
}

vtm_status vtm_set_waves(vtm_handle h, const double *a, int32_t nrhs) {
    if (!h || !a || nrhs < 1) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->set_up) return fail(VTM_ERR_STATE, "no setup");
    HIP_TRY(hipSetDevice(h->opt.device));
    return h->fp32() ? waves_io<float>(h, nullptr, a, nrhs) : waves_io<double>(h, nullptr, a, nrhs);
}

vtm_status vtm_debug_class(vtm_handle h, int32_t k, int64_t *sizes, int32_t *perm, int32_t *sn, int32_t *lev_c0,
                           uint16_t *ridx, uint16_t *rel, int32_t *sc) {
    if (!h || !sizes) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->partitioned || k < 0 || k >= h->P.nsub) return fail(VTM_ERR_STATE, "no partition or k out of range");
    const vtm::ClassSym &C = h->S.classes[h->S.sub_class[k]];
    sizes[0] = C.nk; sizes[1] = C.nsn; sizes[2] = C.nlev; sizes[3] = (int64_t)C.ridx.size();
    sizes[4] = (int64_t)C.sc_src.size(); sizes[5] = C.nval; sizes[6] = C.ws_u; sizes[7] = h->S.sub_class[k];
    if (perm) std::copy(C.perm.begin(), C.perm.end(), perm);
    if (sn)
        for (int32_t s = 0; s < C.nsn; ++s) {
            int32_t *r = sn + 10 * s;
            r[0] = C.sn_c0[s]; r[1] = C.sn_nc[s]; r[2] = C.sn_m[s]; r[3] = C.sn_val[s];
            r[4] = C.sn_ridx[s]; r[5] = C.sn_parent[s]; r[6] = C.sn_level[s]; r[7] = C.sn_uoff[s];
            r[8] = C.sc_ptr[s]; r[9] = C.sc_ptr[s + 1];
        }
    if (lev_c0) std::copy(C.lev_c0.begin(), C.lev_c0.end(), lev_c0);
    if (ridx) std::copy(C.ridx.begin(), C.ridx.end(), ridx);
    if (rel) std::copy(C.rel.begin(), C.rel.end(), rel);
    if (sc)
        for (size_t i = 0; i < C.sc_src.size(); ++i) { sc[2 * i] = C.sc_src[i]; sc[2 * i + 1] = C.sc_dst[i]; }
    return VTM_OK;
}

vtm_status vtm_autotune(vtm_handle h, int32_t nrhs, int32_t *chosen) {
    if (!h || nrhs < 1) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->set_up) return fail(VTM_ERR_STATE, "vtm_autotune before vtm_setup");
    HIP_TRY(hipSetDevice(h->opt.device));
    int32_t maxR = 1;
    while (maxR < nrhs && maxR < 8) maxR *= 2;
    const vtm_options saved = h->opt;
    double best = 1e300;
    vtm_options bestopt = saved;
    Events ev;
    HIP_TRY(ev.create(2));
    const hipEvent_t e0 = ev[0], e1 = ev[1];
    struct Cand { int32_t mode, var, nt; };
    std::vector<Cand> cands;
    for (int32_t var = 1; var <= 2; ++var)
        for (int32_t nt : {128, 256, 512}) cands.push_back({1, var, nt});
    if (h->have_green) cands.push_back({2, 0, 256});
    for (int32_t R = 1; R <= maxR; R *= 2)
        for (const Cand &cd : cands) {
            const size_t lds = cd.mode == 2 ? vtm::schur_lds_bytes(h->tsize(), h->max_p, h->max_np, R, h->opt.sweep_waves)
                             : h->tsize() * (size_t)R * (2 * (size_t)h->max_nk + (cd.var == 2 ? h->max_nu : 0));
            if (lds > 160 * 1024) continue;
            h->opt.rhs_per_block = R;
            h->opt.sweep_threads = cd.nt;
            h->opt.sweep_variant = cd.mode == 2 ? saved.sweep_variant : cd.var;
            h->opt.sweep_mode = cd.mode;
            h->opt.graph_mode = 1;
            vtm_status rc = h->fp32() ? ensure_waves<float>(h, nrhs) : ensure_waves<double>(h, nrhs);
            if (!rc) rc = h->fp32() ? alloc_solve<float>(h, nrhs) : alloc_solve<double>(h, nrhs);
            if (rc) { h->opt = saved; return rc; }
            const int32_t ng = (nrhs + R - 1) / R;
            HIP_TRY(hipMemsetAsync(h->d_bsplit.p, 0, h->tsize() * (size_t)ng * h->nsplit * R, h->stream));
            if (cd.mode == 2) {
                HIP_TRY(ensure(h->d_cport, h->tsize() * ((size_t)ng * h->npg * R + 1)));
                HIP_TRY(hipMemsetAsync(h->d_cport.p, 0, h->tsize() * ((size_t)ng * h->npg * R + 1), h->stream));
            }
            const int64_t warm = 2, timed = 6;
            rc = h->fp32() ? run_sweeps_dev<float>(h, warm) : run_sweeps_dev<double>(h, warm);
            HIP_TRY(hipEventRecord(e0, h->stream));
            if (!rc) rc = h->fp32() ? run_sweeps_dev<float>(h, timed) : run_sweeps_dev<double>(h, timed);
            HIP_TRY(hipEventRecord(e1, h->stream));
            HIP_TRY(hipEventSynchronize(e1));
            if (!rc) rc = check_abort(h);
            if (rc) { h->opt = saved; return rc; }
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bestopt = h->opt;
            }
        }
    h->opt = saved;
    h->opt.rhs_per_block = bestopt.rhs_per_block;
    h->opt.sweep_threads = bestopt.sweep_threads;
    h->opt.sweep_variant = bestopt.sweep_variant;
    h->opt.sweep_mode = bestopt.sweep_mode;
    h->wave_nrhs = 0;  // zero waves for the next solve
    if (chosen) {
        chosen[0] = bestopt.rhs_per_block;
        chosen[1] = bestopt.sweep_threads;
        chosen[2] = bestopt.sweep_variant;
        chosen[3] = bestopt.sweep_mode;
    }
    return VTM_OK;
}

vtm_status vtm_zfeatures(vtm_handle h, float *out) {
    if (!h || !out) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->partitioned) return fail(VTM_ERR_STATE, "no partition");
    if (h->coupled && !h->feats_ready) return fail(VTM_ERR_STATE, "features need the EVS pieces: vtm_setup first");
    ensure_features(h);
    std::copy(h->feats.begin(), h->feats.end(), out);
    return VTM_OK;
}

vtm_status vtm_zmodel_load(vtm_handle h, const void *weights, size_t bytes) {
    if (!h || !weights) return fail(VTM_ERR_INVALID, "bad argument");
    static_assert(vtm::kParams == VTM_ZMODEL_PARAMS && vtm::kTrain == VTM_ZMODEL_TRAIN &&
                      vtm::kNumFeatures == VTM_NUM_FEATURES, "model sizes in vtm.h");
    if (bytes != sizeof(float) * (size_t)vtm::kParams)
        return fail(VTM_ERR_INVALID, "model blob has " + std::to_string(bytes) + " bytes, expected " +
                                         std::to_string(sizeof(float) * (size_t)vtm::kParams));
    std::vector<float> blob(vtm::kParams);
    std::memcpy(blob.data(), weights, bytes);  // the caller's blob need not be aligned
    const float *params = blob.data();
    if (h->host_only()) return fail(VTM_ERR_STATE, "host-only handle");
    for (int i = 0; i < vtm::kParams; ++i)
        if (!std::isfinite(params[i])) return fail(VTM_ERR_INVALID, "non-finite model parameter");
    for (int i = 0; i < vtm::kNumFeatures; ++i)
        if (!(params[vtm::kNumFeatures + i] > 0.f)) return fail(VTM_ERR_INVALID, "feature std must be > 0");
    HIP_TRY(hipSetDevice(h->opt.device));
    std::vector<float> p(params, params + vtm::kParams);
    HIP_TRY(upload(h->d_zparams, p, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->model_loaded = true;
    return VTM_OK;
}

vtm_status vtm_get_z(vtm_handle h, double *z) {
    if (!h || !z) return fail(VTM_ERR_INVALID, "bad argument");
    if (!h->set_up) return fail(VTM_ERR_STATE, "no setup");
    HIP_TRY(hipSetDevice(h->opt.device));
    HIP_TRY(hipMemcpy(z, h->d_z.p, sizeof(double) * h->P.vtl_v.size(), hipMemcpyDeviceToHost));
    return VTM_OK;
}

vtm_status vtm_get_stats(vtm_handle h, vtm_stats *out) {
    if (!h || !out) return fail(VTM_ERR_INVALID, "bad argument");
    *out = h->stats;
    return VTM_OK;
}

}  // extern "C"
