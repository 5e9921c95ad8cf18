// Internal host-side data structures of libvtm.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "vtm.h"

namespace vtm {

// Symmetric input matrix (CSR, both triangles).
struct Csr {
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
};

// EVS partition (Section 4): membership, local pieces, VTLs and ports.
struct Partition {
    int64_t n = 0;
    int32_t nsub = 0;
    std::vector<int64_t> s_ptr;            // membership S(v)
    std::vector<int32_t> s_idx;
    std::vector<int64_t> loc_ptr, loc_vtx;  // vertices of each subgraph, ascending global id
    std::vector<int64_t> lrp;               // local pieces as CSR over local indices
    std::vector<int32_t> lcol;
    std::vector<double> lval;
    std::vector<int64_t> vtl_v;             // VTLs ordered by (v, k, k2), k < k2
    std::vector<int32_t> vtl_k, vtl_k2;
    std::vector<int64_t> port_ptr;          // ports per subgraph ordered by (v, other end)
    std::vector<int64_t> port_v, port_twin, port_vtl;
    std::vector<int32_t> port_other, port_lidx;
    std::vector<double> adiag;              // original diagonal a_vv
    std::vector<double> zdiag;              // Z = 1 / a_vv per VTL
    std::vector<double> coords;             // n x dim vertex coordinates for the local orderings (may be empty)
    int32_t dim = 0;
    int32_t nsys = 1;
    std::vector<int64_t> sys_ptr;           // vertex ranges of independent systems
    std::vector<int32_t> sub_sys;           // system of each subgraph
    uint64_t rcb_seed = 0;                  // RCB: the seed whose boxes met the owned-size bounds
};

int build_partition(const Csr &A, const vtm_partition_spec &spec, Partition &P, std::string &err);

constexpr int kNumFeatures = 13;
// Per-VTL features of the learned impedance model, [nvtl][kNumFeatures].
void compute_features(const Csr &A, const Partition &P, std::vector<float> &out);

// Symbolic analysis of one local sparsity structure ("class"): nested-dissection
// ordering, supernodes sorted by assembly-tree level, multifrontal assembly data
// and the solve layout.  Every subgraph with the same local CSR structure shares it.
struct ClassSym {
    int32_t nk = 0;
    std::vector<int32_t> perm;   // factor position -> local index
    std::vector<int32_t> ipos;   // local index -> factor position
    int32_t nsn = 0, nlev = 0;
    std::vector<int32_t> sn_c0, sn_nc, sn_m, sn_val, sn_ridx, sn_parent, sn_level, sn_uoff;
    std::vector<int32_t> lev_c0;     // column range of each level (nlev + 1)
    std::vector<int32_t> lev_maxf;   // largest front order nc + m of each level (nlev + 1, last 0)
    std::vector<int32_t> col_sn;     // supernode of each factor column
    std::vector<uint16_t> ridx;      // R_s rows (factor positions), concatenated
    std::vector<uint16_t> rel;       // position of each R_s row inside the parent's front
    std::vector<int32_t> ch_ptr, ch_idx;  // children of each supernode
    std::vector<int32_t> colrec;     // per factor column: {block offset, c0<<16|nc, jj<<16|m, ridx offset}
    std::vector<int32_t> urec;       // per update entry (row nc + q of its supernode): same four fields
    std::vector<uint16_t> u_sn;      // supernode of every update entry (one per R_s row, ridx order)
    std::vector<uint16_t> seg_u;     // update entries summed into each factor row (CSR by seg_ptr)
    std::vector<int32_t> lev_u;      // update-entry range of each level (nlev + 1)
    std::vector<int32_t> seg_ptr;    // forward-solve segments of each factor row
    std::vector<int32_t> seg_off;    // value offset of the L21 row of the segment
    std::vector<uint16_t> seg_c0, seg_nc;
    std::vector<int32_t> sc_ptr, sc_src, sc_dst;  // assembly: local CSR entry -> front position
    int64_t nval = 0;                // stored factor values per subgraph
    int64_t nlower = 0;              // stored lower-triangular entries actually used by the solve
    int64_t ws_u = 0;                // update-matrix workspace per subgraph
    int32_t max_front = 0;           // largest front order nc + m
    int64_t nnz_local = 0;           // entries of the local CSR
};

struct Symbolic {
    std::vector<int32_t> sub_class;
    std::vector<ClassSym> classes;
};

int build_symbolic(const Partition &P, int leaf, Symbolic &S, std::string &err);

}  // namespace vtm
