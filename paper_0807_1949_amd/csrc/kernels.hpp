// Device data views and kernel launchers of libvtm (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vtm {

// Per-class symbolic data: offsets into the concatenated class arrays.
struct ClassDev {
    int32_t nk, nsn, nlev, max_front;
    int32_t o_lev;   // lev_c0        (nlev + 1 per class)
    int32_t o_sn;    // sn_* arrays   (nsn per class)
    int32_t o_snp;   // ch_ptr, sc_ptr (nsn + 1 per class)
    int32_t o_col;   // col_sn        (nk per class)
    int32_t o_colp;  // seg_ptr       (nk + 1 per class)
    int32_t o_ridx;  // ridx, rel
    int32_t o_seg;   // seg_off, seg_c0, seg_nc
    int32_t o_sc;    // sc_ptr entries of the class (assembly scatter list)
    int32_t o_chi;   // ch_idx
    int32_t nu;      // update entries (sum of m over supernodes)
    int64_t nval, ws_u;
};

struct DevSym {
    const ClassDev *cls;
    const int32_t *lev_c0, *col_sn;
    const int32_t *lev_maxf;        // largest front of each level (lev offsets)
    const int32_t *sn_c0, *sn_nc, *sn_m, *sn_val, *sn_ridx, *sn_uoff;
    const uint16_t *ridx, *rel;
    const int32_t *ch_ptr, *ch_idx;
    const int32_t *seg_ptr, *seg_off;
    const uint16_t *seg_c0, *seg_nc;
    const uint16_t *seg_u, *u_sn;   // update-entry lists (variant 1 of the sweep)
    const int32_t *colrec, *urec;   // per column and per update entry: {block offset, c0<<16|nc, row<<16|m, ridx offset}
    const int32_t *lev_u;           // update-entry range per level (lev offsets)
    const int32_t *sc_ptr, *sc_dst;
};

struct DevSub {
    const int32_t *cls;
    const int64_t *val;   // factor value offset
    const int64_t *x;     // offset of the subgraph's entries in split vectors (factor order)
    const int64_t *aval;  // offset of the subgraph's assembly values (lower local entries, scatter order)
    const int64_t *ws;    // factorisation workspace offset
    const int32_t *pg_ptr;   // port groups of each subgraph (nsub + 1)
    const uint16_t *pg_pos;  // factor position of the group's vertex
    const int32_t *pg_beg;   // first port of the group
    const int32_t *pg_cnt;   // ports in the group
    const int32_t *port_ptr; // first port of each subgraph (nsub + 1)
    const uint16_t *port_pg; // port -> index of its port vertex (group) in its subgraph
    const int32_t *gorder;   // subgraphs by decreasing size of G_k (launch order of the port-reduced sweep)
    const int32_t *sub_sys;  // independent system of each subgraph
    const int32_t *active;   // per system: 0 once it has converged (its subgraphs skip sweeps and test
                             // solves); nullptr = every system active
    // coupled VTLs: per port p, entries [cpl_ptr[p], cpl_ptr[p + 1]) name the twin of each other port q
    // of its subgraph coupled with it and (Z_j^{-1})_pq; cpl_ptr == nullptr when Z is diagonal
    const int32_t *cpl_ptr;
    const int32_t *cpl_tw;
    const double *cpl_y64;
    const float *cpl_y32;
    // the subgraphs a launch covers (done mask: those of the systems still sweeping, largest G_k first),
    // one per workgroup; nullptr = every subgraph (gorder for the port-reduced sweep, else by id)
    const int32_t *sub_list;
};

// Subgraph of workgroup b: from the launch list, else in the given default order.
__device__ inline int sub_of_block(const DevSub &D, int b) { return D.sub_list ? D.sub_list[b] : b; }

// Skip the workgroups of converged systems (done mask of a batched solve).
__device__ inline bool sub_inactive(const DevSub &D, int k) { return D.active && !D.active[D.sub_sys[k]]; }

// Column plan of the port Green's functions computed inside the factorisation.  Ports of a subgraph
// are sorted by the postorder of their supernode, so the ports below supernode s form one column
// range [pc0, pc0 + w) and a child's range lies inside its parent's.  Plan entries of subgraph k
// start at base[k] (one per supernode).  sn == nullptr: no Green's functions.
struct DevGreen {
    const int4 *sn;         // {port-front offset, pc0 | w << 16, parent's port-front offset, parent pc0 | parent w << 16}
    const int32_t *base;    // first plan entry of each subgraph
    const int64_t *wso;     // workspace offset of each subgraph (doubles)
    const int32_t *idoff;   // per sorted port: workspace offset of its unit right-side entry
    const uint16_t *perm;   // per sorted port: its port-vertex index in the subgraph
    double *ws;             // port fronts (nc + m) x w followed by Y blocks nc x w; zero on entry
    float *ws32;            // FP32 copy of the Y blocks (same regions, rows padded to 4 when w >= 4), or nullptr
};

// Split-vector and merge maps.
struct DevMaps {
    const int32_t *fvtx;   // split entry (factor order) -> global vertex
    const int32_t *fmul;   // |S(v)| of that vertex
    const int64_t *cp_ptr; // vertex -> its split entries
    const int32_t *cp_idx;
};

struct DevCsr {
    const int64_t *rp;
    const int32_t *ci;
    const double *v;
};

void launch_invz(const double *z_vtl, const int32_t *port_vtl, double *invz64, float *invz32, int64_t nports,
                 hipStream_t st);

// FP64 multifrontal factorisation of every port-augmented local matrix; status[k] = 1 + supernode of the
// first non-positive pivot (0 if fine).  With Gp.sn set it also computes the port Green's columns Y_s
// and, when G is given, accumulates G_k = R K_k^{-1} R^T (FP64, packed lower block triangle at goff[k],
// see k_schur; zero on entry); with G == nullptr launch_gram forms G_k afterwards.
void launch_factor(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_front, const double *aval,
                   const double *invz, double *vals, float *vals32, double *ws, int32_t *status, const DevGreen &Gp,
                   const int64_t *goff, double *G, hipStream_t st);

// G_k = sum_s Y_s^T Y_s from the Y blocks a factorisation left in Gp.ws (launched after launch_factor
// with G == nullptr, which then skips these products); every stored entry of G is written.  Needs
// G_k's port order to be the plan order (Gp.perm the identity).
void launch_gram(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_p, const DevGreen &Gp,
                 const int64_t *goff, double *G, hipStream_t st);

void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t st);

// The solver's FP64 n-vectors (right sides, iterates, residuals) are row-interleaved: the nrhs values
// of vertex v at v * S .. v * S + nrhs, with the row stride S padded to a multiple of four beyond two
// (whole 32-byte rows for the residual's loads), padding zero.  The residual takes res_group(S)
// columns per pass.
inline int32_t vec_stride(int32_t nrhs) { return nrhs <= 2 ? nrhs : (nrhs + 3) & ~3; }
inline int32_t res_group(int32_t S) { return S <= 2 ? S : S % 8 == 0 ? 8 : 4; }

// Rows of the systems flagged in flag[] (per system) moved between the solve's two iterate buffers,
// by residual chunks: 1 copies x from xb to xa, 2 also r from rb to ra, 3 copies x from xa to xb.
void launch_sys_rows(const int64_t *chunk_row, const int32_t *chunk_sys, int32_t nchunks, const int32_t *flag,
                     int32_t S, double *xa, double *xb, double *ra, const double *rb, hipStream_t st);

// Column-major n x nrhs (leading dimension ld) to row-interleaved rows of stride S, and back.
void launch_to_rows(const double *src, int64_t ld, int64_t n, int32_t nrhs, int32_t S, double *dst, hipStream_t st);
void launch_from_rows(const double *src, int32_t S, int64_t n, int32_t nrhs, double *dst, int64_t ld, hipStream_t st);

// bsplit[g][e][cc] = b[fvtx[e]][g R + cc] / |S(v)| (source split; b row-interleaved, stride S).
template <typename T>
void launch_split(const DevMaps &M, int64_t nsplit, const double *b, int32_t nrhs, int32_t S, int32_t R,
                  T *bsplit, hipStream_t st);

// Restart of the inner solves of some systems (iterative refinement, one system at a time): for the
// nlist subgraphs of D.sub_list (of nsub), the source split of the new right side b and zero outgoing waves on
// their ports in o (the buffer the next sweep reads).
template <typename T>
void launch_restart(const DevSub &D, const DevMaps &M, int32_t nsub, int32_t nlist, int64_t nsplit, int64_t nports,
                    const double *b, int32_t nrhs, int32_t S, int32_t R, T *bsplit, T *o, hipStream_t st);

// LDS bytes the substitution sweep needs for one right-hand side (largest local system and update
// workspace); more than kMaxLds cannot run.
size_t sweep_lds_min(size_t tsize, int32_t max_nk, int32_t max_nu);

// One VTM sweep over all subgraphs and right-hand-side groups (grid = subgraphs x RHS groups).
template <typename T>
void launch_sweep(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_nk, int32_t max_nu, int32_t variant,
                  int32_t ngroups, int32_t R, int32_t threads, int64_t nsplit, int64_t nports, const T *vals, const T *bsplit, const int32_t *twin,
                  const T *invz, const T *o_prev, T *o_next, T *xloc, T *yout, int flags, hipStream_t st);
constexpr int kSweepWriteX = 1, kSweepNoWaves = 2, kSweepZeroWaves = 4, kSweepWriteY = 8;  // sweep flags
// Raise the dynamic-LDS limit of the sweep kernel when needed (call outside stream capture).
template <typename T>
hipError_t prepare_sweep(int32_t max_nk, int32_t max_nu, int32_t variant, int32_t R);

// Local solutions of a convergence test from the stored Y blocks (Yw: the Green workspace in T
// precision) and y_b = L^{-1} b~ (yb, layout of the local solutions): one parallel product and the
// backward substitution, `threads` (64 .. 512) per subgraph.  prepare_ysolve fails when the LDS need
// exceeds the CU's.
template <typename T>
hipError_t prepare_ysolve(int32_t max_nk, int32_t max_p, int32_t R);
template <typename T>
void launch_ysolve(const DevSym &S, const DevSub &D, const DevGreen &Gp, const T *Yw, int32_t nsub, int32_t max_nk,
                   int32_t max_p, int32_t ngroups, int32_t R, int32_t threads, int64_t nsplit, int64_t nports,
                   const T *vals, const T *yb, const int32_t *twin, const T *invz, const T *o_in, T *xloc,
                   hipStream_t st);

// Port Green's functions G_k = R K_k^{-1} R^T by one substitution per group of four port columns
// (FP64, packed like above); used when the column plan does not apply.
void launch_green(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_nk, int32_t max_nu, int32_t max_p,
                  const double *vals, const int64_t *goff, double *G, hipStream_t st);
// gd[port vertex] = diagonal entry of its G_k (FP64).
void launch_gdiag(const DevSub &D, int32_t nsub, const int64_t *goff, const double *G, double *gd, hipStream_t st);
// r[port] = input impedance of the port (Definition 7.1, other ports terminated) from the FP64 G_k.
void launch_rin(const DevSub &D, int32_t nsub, const int64_t *goff, const double *G, const double *invz, double *r,
                hipStream_t st);
// Scratch of the allocation-free entry points: kNoAllocDoubles doubles per device in a file-scope device
// array; *ptr = its address on `device`, which must be current (looked up once per device, then cached).
constexpr size_t kNoAllocDoubles = (size_t)1 << 22;  // 32 MiB
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, double **ptr);
// cport[g][port vertex][R] = local solutions at the port vertices.
template <typename T>
void launch_gather_ports(const DevSub &D, int32_t nsub, int32_t ngroups, int64_t nsplit, int32_t npg, int32_t R,
                         const T *xloc, T *cport, hipStream_t st);
template <typename T>
hipError_t prepare_schur(int32_t max_p, int32_t max_np, int32_t R, int32_t W);
// Waves per subgraph of the port-reduced sweep (W = 0: chosen from the LDS size) and its LDS; it
// runs only when this fits the 160 KiB of a CU.
int32_t schur_waves(size_t tsize, int32_t max_p, int32_t max_np, int32_t R, int32_t W);
size_t schur_lds_bytes(size_t tsize, int32_t max_p, int32_t max_np, int32_t R, int32_t W = 0);
constexpr size_t kMaxLds = 160 * 1024;
// Port-reduced sweep: o = 2 (c + G Z^{-1} a) - a at every port.
template <typename T>
void launch_schur(const DevSub &D, int32_t nsub, int32_t ngroups, int32_t R, int32_t W, int32_t max_p, int32_t max_np,
                  int32_t npg, int64_t nports, const T *G, const int64_t *goff, const T *cport, const int32_t *twin,
                  const T *invz, const T *o_prev, T *o_next, hipStream_t st);

// Persistent port-reduced sweeps (FP32, p_k <= 128): nsw sweeps in one cooperative launch, G_k rows in registers,
// waves exchanged as tagged 64-bit words tw[2][ngroups][nports][R] (the launch publishes the plain
// waves plain[cur0] with tag t0 first, then awaits tags t0 .. t0 + nsw - 1, which no word left in tw
// from earlier use may carry); the last two sweeps also write the plain buffers (cur0 ^ (i & 1)).
// *abort_flag becomes 1 if a wait exceeded spin_limit polls.
size_t persist_lds_bytes(int32_t max_p, int32_t max_np, int32_t R);
int persist_max_p();  // largest port-vertex count per subgraph of the persistent kernel
hipError_t persist_capacity(int32_t max_p, int32_t max_np, int32_t R, int64_t *resident);
hipError_t launch_schur_persist(const DevSub &D, int32_t nsub, int32_t ngroups, int32_t R, int32_t max_p,
                                int32_t max_np, int32_t npg, int64_t nports, const float *G, const int64_t *goff,
                                const float *cport, const int32_t *twin, const float *invz, unsigned long long *tw,
                                float *plain0, float *plain1, int32_t t0, int32_t nsw, int32_t cur0,
                                int32_t spin_limit, int32_t *abort_flag, hipStream_t st);

// xout[v][c] = (base ? base[v][c] : 0) + mean over the children of v of xloc (row-interleaved, stride
// S), by residual chunks (chunk_row[nchunks + 1]: row ranges of at most 256 rows inside one system,
// chunk_sys: their systems); the rows of a system with active[s] == 0 are left as they are (active may
// be null).
template <typename T>
void launch_merge(const DevMaps &M, int64_t nsplit, int32_t nrhs, int32_t S, int32_t R, const T *xloc,
                  const double *base, double *xout, const int64_t *chunk_row, const int32_t *chunk_sys,
                  int32_t nchunks, const int32_t *active, hipStream_t st);

// r = b - A x (b, x, r row-interleaved, stride S; optional store of r), per (rhs, system) relative
// residual into relres[c * nsys + s], and
// relres[nsys * nrhs] = 1 if *flag is set (flag may be null), so that one copy brings both to the host.
// Rows of the chunks of a system with active[s] == 0 (active may be null) are skipped; their partial
// sums keep the values of the last pass over them.
void launch_residual(const DevCsr &A, int64_t n, int32_t nrhs, int32_t S, const double *b, const double *x, double *r,
                     const int64_t *chunk_row, const int32_t *chunk_sys, const int32_t *active, int32_t nchunks,
                     const int32_t *sys_chunk_ptr, int32_t nsys, double *part, const int32_t *flag, double *relres,
                     hipStream_t st);

}  // namespace vtm
