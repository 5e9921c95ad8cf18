/*
 * vtm.h -- C ABI of libvtm, a gfx950 (MI355X) implementation of the Virtual
 * Transmission Method (VTM) over an Electric-Vertex-Split (EVS) SPD system,
 * after F. Wei and H. Yang, "Virtual Transmission Method, A New Distributed
 * Algorithm to Solve Sparse Linear System".
 *
 * Problem statement (Section 3, eq. (3.1)): solve A x = b with A sparse,
 * symmetric positive definite.  The library
 *   1. splits the electric graph of A by EVS (Section 4: boundary, twin
 *      children, split weights/sources, ports; multilevel splitting, Fig. 7),
 *   2. agrees on one characteristic impedance Z per virtual transmission line
 *      (VTL) and factors every port-augmented local matrix of eq. (5.8),
 *      C_j + Z_j^{-1} on the ports, once (Table 1 step 1; Section 8),
 *   3. iterates Table 1 steps 3-6: every sweep solves all local systems (5.8)
 *      with the stored factors and exchanges port waves with the twins under
 *      the transmission delay equations (5.6), delay = one sweep.
 * All subdomains live on one GPU; the neighbour-to-neighbour exchange is a
 * gather of outgoing waves by twin index.
 *
 * Conventions (all entry points):
 *   - Every call returns a vtm_status; VTM_OK (0) on success.  No exception
 *     crosses the ABI.  vtm_last_error() returns a thread-local message for the
 *     last failing call on the calling thread.
 *   - Inputs are borrowed for the duration of the call (deep-copied where kept).
 *     Outputs are caller-allocated.
 *   - Matrices are CSR with both triangles stored, sorted column indices, an
 *     explicit positive diagonal: rowptr int64[n+1], col int32[nnz],
 *     val double[nnz], host memory.
 *   - Vectors b and x of vtm_solve / vtm_run_sweeps may be host or device
 *     pointers (detected with hipPointerGetAttributes); column c of an n x nrhs
 *     block starts at ptr + c * ld.
 *   - A handle is not thread-safe; distinct handles may be used from distinct
 *     threads.  All device work of a handle runs on its stream.
 */
#ifndef VTM_H
#define VTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vtm_status;

enum {
    VTM_OK = 0,
    VTM_ERR_INVALID = 1,        /* null / size / non-symmetric / non-finite input, tol <= 0, Z <= 0 */
    VTM_ERR_PARTITION = 2,      /* an edge not inside any subgraph, an empty subgraph, RCB bounds failed */
    VTM_ERR_NOT_SPD = 3,        /* a local pivot <= 0 during factorisation (subdomain in message) */
    VTM_ERR_NOT_CONVERGED = 4,  /* max sweeps reached; x, iters, relres are still written */
    VTM_ERR_DIVERGED = 5,       /* NaN or residual growth > 1e3 x its initial value */
    VTM_ERR_STATE = 6,          /* call order violated (e.g. solve before setup) */
    VTM_ERR_HIP = 7,            /* HIP runtime error */
    VTM_ERR_OOM = 8             /* host or device allocation failed */
};

enum { VTM_FP64 = 0, VTM_FP32_IR = 1 };
enum { VTM_PART_GRID = 0, VTM_PART_RCB = 1, VTM_PART_GRAPH = 2, VTM_PART_USER = 3 };
enum { VTM_SPLIT_BRANCH = 0, VTM_SPLIT_EQUAL = 1 };
enum { VTM_TOPO_FACE = 0, VTM_TOPO_COMPLETE = 1, VTM_TOPO_TREE = 2 };
enum { VTM_Z_DIAG = 0, VTM_Z_USER = 1, VTM_Z_LEARNED = 2, VTM_Z_MATCHED = 3 };

typedef struct vtm_ctx *vtm_handle;

typedef struct {
    int32_t device;        /* HIP device ordinal; -1 = host-only handle (partition and its analysis only) */
    void *stream;          /* hipStream_t to run on; NULL = the library creates its own */
    int32_t precision;     /* VTM_FP64, or VTM_FP32_IR: FP32 factors and sweeps, FP64 refinement */
    int32_t check_every;   /* sweeps between convergence tests; 0 = adaptive (placed where the observed
                              contraction rate predicts the tolerance, 5..200 sweeps apart) */
    int64_t max_sweeps;    /* cap on sweeps per solve (0 = default 100000) */
    int32_t rhs_per_block; /* right-hand sides one workgroup carries (0 = tuned: 1, 2, 4 or 8) */
    int32_t leaf_size;     /* nested-dissection leaf size of the local orderings (0 = 16) */
    int32_t sweep_threads; /* threads per substitution workgroup (sweeps and test solves), 64..512
                              (0 = 256, or vtm_autotune's choice) */
    int32_t graph_mode;    /* 0: replay sweep batches as captured HIP graphs; 1: plain launches */
    int32_t sweep_variant; /* forward substitution: 1 = row dot products over descendant L21 rows,
                              2 = per-level update entries L21*y gathered by the ancestors, 0 = choose */
    int32_t sweep_mode;    /* 1 = substitution sweeps; 2 = port-reduced sweeps u = c + G Z^{-1} a with the
                              port Green's functions G_k = R_k K_k^{-1} R_k^T (same iterates; the
                              substitution runs only at convergence tests); 0 = port-reduced when the packed
                              G_k hold at most 8 times the stored factor entries.
                              Port-reduced sweeps need a subgraph's port vectors in LDS
                              (about 2 p_k rhs_per_block values per wave); when they do not fit,
                              or G_k was not built (p_k > 2048), substitution sweeps run. */
    int32_t persistent;    /* port-reduced FP32 sweeps: 0 = one persistent cooperative launch per batch of
                              sweeps between tests when every workgroup fits on the device at once, each
                              wave's G_k blocks fit in registers and rhs_per_block <= 2 (G_k held on chip,
                              waves exchanged as tagged words), else per-sweep launches;
                              1 = per-sweep launches only */
    int32_t sweep_waves;   /* port-reduced sweeps in per-sweep launches: waves per subgraph, 1 or 2 (two
                              waves take alternate pairs of block columns of G_k, each with its own
                              copy of the products); 0 = two when one wave's LDS would leave fewer than
                              two waves per SIMD, or when the subgraphs still sweeping (done mask) are
                              fewer than two per compute unit */
    int32_t spin_limit;    /* persistent sweeps: polls of one incoming wave word before the launch gives up
                              (every other wait then gives up too, the launch ends, and the solve or
                              vtm_run_sweeps returns VTM_ERR_HIP; the handle stays usable); 0 = 2^20.
                              A small value forces that path (tests of the failure handling) */
} vtm_options;

/*
 * EVS partition scheme (Section 4, steps 1-4; "partition scheme" below
 * Example 4.1).  Membership S(v) = subgraphs holding a child of vertex v:
 *   GRID : vertex grid dims (x fastest); parts[a] tiles per axis sharing their
 *          separator lines: m = dims/parts if exact else (dims-1)/parts, tile I
 *          covers [I*m, (I+1)*m], the last tile ends at dims-1.  Ids row-major.
 *   RCB  : seeded random recursive coordinate bisection of the vertex grid into
 *          2^levels boxes sharing cut planes; longest axis (ties: lowest) cut at
 *          lo + (len*q + 50)/100, q = 49 + splitmix64(state) mod 3, depth-first
 *          pre-order; accepted iff every box's owned size sum 1/|S(v)| lies in
 *          [min_size, max_size], else redrawn from seed + 1, ... (64 seeds; the seed
 *          used is reported in vtm_partition_info.rcb_seed).
 *   GRAPH: per block of vertices (an independent system), point RCB on coords
 *          into block_parts[b] owners; every cut edge (u,v) with
 *          owner(u) < owner(v) adds owner(v) to S(u).
 *   USER : S(v) given as sorted lists s_idx[s_ptr[v] .. s_ptr[v+1]).
 * Weights (step 3): split_rule BRANCH gives every piece of an edge
 * a_uv / |S(u) & S(v)| and every child of v the sum of its branch magnitudes
 * plus an equal share of a_vv - sum_u |a_uv| (weakly diagonally dominant
 * pieces, hence SNND -- Corollary 4.1 -- for M-matrices); EQUAL gives a_vv/|S(v)|.
 * Sources are split b_v / |S(v)|.  Multilevel splitting (Fig. 7): topology FACE
 * joins two children of v by a VTL iff their subgraphs share a vertex of
 * multiplicity 2 somewhere (all pairs if that leaves S(v) disconnected);
 * COMPLETE joins all pairs; TREE keeps of the FACE pairs, taken in (k, k') order, those
 * that join two children not yet connected -- the |S(v)| - 1 VTLs of splitting v again and
 * again into two (no cycle of VTLs at one vertex, around which waves could circulate).
 */
typedef struct {
    int32_t kind;
    int32_t dims[3];
    int32_t parts[3];
    int32_t levels;
    uint64_t seed;
    double min_size, max_size;
    const double *coords;        /* n x dim row-major (GRAPH; optional for USER) */
    int32_t dim;
    int32_t nblocks;
    const int64_t *block_start;  /* GRAPH: first vertex of each block */
    const int64_t *block_count;  /* GRAPH: vertices in each block */
    const int32_t *block_parts;  /* GRAPH: subgraphs per block */
    const int64_t *s_ptr;        /* USER */
    const int32_t *s_idx;        /* USER */
    int32_t user_nsub;           /* USER */
    int32_t split_rule;
    int32_t topology;
    int32_t nsys;                /* independent systems for per-system convergence (0/1 = one) */
    const int64_t *sys_ptr;      /* nsys+1 vertex offsets of the systems (NULL if nsys <= 1) */
} vtm_partition_spec;

typedef struct {
    int32_t nsub;            /* subgraphs N */
    int32_t nclass;          /* distinct local sparsity structures (shared symbolic analysis) */
    int64_t n_split;         /* unknowns after splitting, sum of |M_j| */
    int64_t nvtl;            /* virtual transmission lines */
    int64_t nports;          /* ports (2 per VTL) */
    int32_t max_local;       /* largest |M_j| */
    int32_t nsys;            /* independent systems */
    int64_t factor_entries;  /* stored factor entries over all subgraphs */
    uint64_t rcb_seed;       /* RCB: the seed actually used (seed, seed + 1, ... until the bounds hold) */
} vtm_partition_info;

typedef struct {
    int64_t sweeps;          /* sweeps of the last solve (all outer steps) */
    int32_t outer_steps;     /* refinement steps of the last solve (FP32_IR; the most any one system took), 1 in FP64 */
    int32_t checks;          /* convergence tests of the last solve */
    double setup_ms;         /* last vtm_setup: Z, augmentation and factorisation (device time) */
    double solve_ms;         /* last solve, wall time on the stream (events) */
    double sweep_ms;         /* last solve, summed sweep-kernel time (events around sweep launches) */
    double bytes_per_sweep;  /* algorithmic bytes per sweep: factor (substitution) or G (port-reduced; in
                                persistent launches read once per launch, so averaged over its sweeps)
                                + vectors + waves */
    double flops_per_sweep;  /* substitution: 4 * nrhs * lower-factor entries; port-reduced: 2 * nrhs * G entries */
    int32_t sweep_mode;      /* mode of the last solve or vtm_run_sweeps: 1 substitution, 2 port-reduced */
    int32_t persistent;      /* 1 if the last solve or run ran its sweeps in persistent launches */
    double sweep_bytes;      /* last solve: algorithmic bytes of all its sweeps, counting only the systems
                                still sweeping (done mask) and G once per persistent launch */
} vtm_stats;

/* Create a handle bound to options->device; NULL options = defaults. */
vtm_status vtm_create(const vtm_options *options, vtm_handle *out);
/* Release every host and device resource of the handle. */
vtm_status vtm_destroy(vtm_handle h);
/* Message of the last failing call on this thread ("" if none). */
const char *vtm_last_error(void);

/*
 * EVS partition of A (host CSR, see conventions) following spec; builds the
 * local pieces, VTLs, ports and twins, and the per-class symbolic analysis of
 * the local factors (nested dissection ordering, supernodes).  Replaces any
 * previous partition of the handle.  No device work besides uploads.
 * Errors: VTM_ERR_INVALID (bad CSR or spec), VTM_ERR_PARTITION.
 */
vtm_status vtm_evs_partition(vtm_handle h, int64_t n, const int64_t *rowptr, const int32_t *col,
                             const double *val, const vtm_partition_spec *spec, vtm_partition_info *info);

/*
 * Copy the partition out (host arrays sized from vtm_partition_info; any may be
 * NULL).  Layouts match the description in vtm_evs_partition:
 *   s_ptr[n+1], s_idx[*]          membership, sorted per vertex
 *   loc_ptr[nsub+1], loc_vtx[n_split]   vertices of each subgraph, ascending
 *   lrp[n_split+1], lcol[*], lval[*]    local pieces A~_k as CSR over local indices
 *   vtl_v, vtl_k, vtl_k2 [nvtl]   VTLs ordered by (v, k, k'), k < k'
 *   port_ptr[nsub+1], port_v[nports], port_other[nports], port_twin[nports]
 *                                 ports of each subgraph ordered by (v, other end)
 *   zdiag[nvtl]                   the diagonal rule Z = 1 / a_vv
 */
vtm_status vtm_get_partition(vtm_handle h, int64_t *s_ptr, int32_t *s_idx, int64_t *loc_ptr, int64_t *loc_vtx,
                             int64_t *lrp, int32_t *lcol, double *lval, int64_t *vtl_v, int32_t *vtl_k,
                             int32_t *vtl_k2, int64_t *port_ptr, int64_t *port_v, int32_t *port_other,
                             int64_t *port_twin, double *zdiag);

/*
 * Table 1 step 1 and eq. (5.8): set one impedance per VTL and factor every
 * port-augmented local matrix K_k = A~_k + sum_{p in k} Z_p^{-1} e_v(p) e_v(p)^T
 * on the device (multifrontal Cholesky; diagonal blocks stored inverted).
 *   z_rule VTM_Z_DIAG   : Z = 1 / a_vv (z_vtl ignored)
 *          VTM_Z_USER   : z_vtl[nvtl] host array, finite and > 0
 *          VTM_Z_LEARNED: the loaded impedance model predicts ln(Z a_vv) per VTL
 *                         (vtm_zmodel_load first); z_vtl ignored
 *          VTM_Z_MATCHED: impedance matching (Section 7.1): starting from 1/a_vv, twice
 *                         set each VTL's Z to the geometric mean of its two ports' input
 *                         impedances (vtm_input_impedance), kept within [1/4, 4096] / a_vv,
 *                         and factor again; needs at most 2048 port vertices per subgraph
 *                         (else VTM_ERR_INVALID); setup_ms covers all three factorisations
 * Resets the waves to zero.  Errors: VTM_ERR_STATE (no partition),
 * VTM_ERR_INVALID (Z; or a subgraph too large for a local solve: its vectors, 2 n_k + the largest
 * update workspace values, must fit one CU's 160 KiB of LDS), VTM_ERR_NOT_SPD (first failing
 * subgraph in the message).
 */
vtm_status vtm_setup(vtm_handle h, int32_t z_rule, const double *z_vtl);

/*
 * Coupled VTLs (Section 7.2, Theorem 7.1): the local preconditioner Z_j of (5.6)-(5.8) is an SPD matrix
 * over the ports of a subgraph instead of a diagonal one.  Z is given as a symmetric matrix over the
 * VTLs: diagonal z_vtl[nvtl] (> 0) and the off-diagonal entries Z[vtl_a[e]][vtl_b[e]] = z_ab[e],
 * e < ncouple, each unordered pair at most once (host arrays).  Coupled VTLs must join the same two
 * subgraphs; Z is then block diagonal over groups of VTLs between one pair of subgraphs, and both
 * subgraphs of a group use its block, in their own port order, as their Z_j, so that the twins of
 * (5.6) see the same matrix.  Every block must be positive definite (Theorem 7.1's condition).
 * The local matrix of (5.8) gets the block Z_j^{-1} on the group's port vertices (which may add
 * entries to a local sparsity pattern; the symbolic analysis is redone), every sweep adds
 * Z_j^{-1} a to the right side, and the outgoing waves stay o = u - Z_j w = 2u - a with
 * w = Z_j^{-1}(a - u).  Sweeps run as substitution sweeps (no port Green's functions), in the
 * handle's precision; vtm_solve / vtm_run_sweeps / waves calls work as after vtm_setup.  A later
 * vtm_setup returns to diagonal impedances (and the original analysis).  vtm_get_partition keeps
 * returning the EVS pieces.  vtm_batch_solve does not take coupled members.
 * Errors: VTM_ERR_STATE (no partition), VTM_ERR_INVALID (an entry out of range or non-finite, coupled
 * VTLs between different subgraph pairs, a block not positive definite), VTM_ERR_NOT_SPD.
 */
vtm_status vtm_setup_coupled(vtm_handle h, const double *z_vtl, int64_t ncouple, const int64_t *vtl_a,
                             const int64_t *vtl_b, const double *z_ab);

/*
 * Definition 7.1: the input impedance of every port, i.e. its potential for a unit inflow current
 * there, with every other port of its subgraph terminated by its current characteristic impedance
 * (as Z grows the terminations vanish and this tends to the definition's value with the other ports
 * open, which needs an SPD piece).  From the port Green's functions of the last vtm_setup: with g
 * the diagonal entry of R K_k^{-1} R^T at the port's vertex, r = 1 / (1/g - 1/Z_p); +inf where the
 * port's own termination is what makes K_k definite.
 *   r_port[nports]: host array, ports in partition order.
 * Errors: VTM_ERR_STATE (no setup, or the setup built no Green's functions: sweep_mode 1 or more
 * than 2048 port vertices in a subgraph).
 */
vtm_status vtm_input_impedance(vtm_handle h, double *r_port);

/*
 * vtm_input_impedance for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same values, computed on the device
 * into a fixed scratch of 2^22 doubles (32 MiB) that each GPU the library runs on holds until the
 * process ends; no hipMalloc, hipFree or allocating call.  r_port[nports] may be a host or a device
 * pointer.  More than 2^22 ports: VTM_ERR_INVALID.  Every call on one GPU uses that GPU's scratch,
 * so calls that overlap on one GPU (from several threads or streams) race; the scratch keeps the last
 * call's values and every entry the call returns is written by it.  Errors as vtm_input_impedance.
 */
vtm_status vtm_input_impedance_noalloc(vtm_handle h, double *r_port);

/*
 * Solve A X = B for nrhs right-hand sides: zero initial waves (Example 5.1),
 * sweeps until every system's relative residual ||b - A xbar||_2 / ||b||_2 is
 * <= tol for every column, where xbar_v is the mean of the children of v
 * (tested every check_every sweeps).  FP32_IR runs FP32 sweeps on the
 * correction equation and refines x in FP64.
 *   b: n x nrhs (ld >= n), host or device;  x: n x nrhs output (ldx >= n)
 *   iters[nrhs*nsys]: first passing sweep per (rhs, system), -1 if none; index c * nsys + s
 *   relres[nrhs*nsys]: relative residual of the returned x
 * With several systems (vtm_partition_spec.nsys > 1) a system whose right-hand sides all pass
 * stops sweeping (its x is kept) while the others go on; in FP32_IR each system also restarts its
 * inner solve on its own new residual (after a gain of 1e-5 or a stall; a system that stalls
 * without improving stops, and the call then returns VTM_ERR_NOT_CONVERGED).  Test placement
 * (check_every = 0) depends on the residual history only, so sweep counts repeat from run to run.
 * Returns VTM_ERR_NOT_CONVERGED (with outputs written) if max_sweeps is hit,
 * VTM_ERR_DIVERGED on NaN or growth.
 */
vtm_status vtm_solve(vtm_handle h, const double *b, int32_t nrhs, int64_t ldb, double tol, double *x, int64_t ldx,
                     int32_t *iters, double *relres);

/*
 * Many independent systems (the problem statement of Section 3 for each handle) solved together:
 * the members' subgraphs run in one launch per sweep, each member's systems keep their own
 * convergence test (Table 1 step 6), and a system whose right-hand sides all pass stops sweeping
 * while the others go on (done mask).  Members must be set up, on one device, with one precision;
 * the batch runs with the options and on the stream of hs[0].  The first call for a list of members
 * (and the first after any member's vtm_setup) builds the batch: it copies the members'
 * partitions, analyses and impedances into a context owned by hs[0] and factors them there again
 * (the members' own factors and waves are not used or changed); later calls reuse it.
 *   hs[count]; b[i], x[i]: n_i x nrhs blocks (host or device) with leading dimensions ldb[i], ldx[i]
 *   iters[i], relres[i] (either array or any entry may be NULL): [nrhs * nsys_i] as in vtm_solve
 * Every member's statistics become those of the batch solve.  Errors as vtm_solve, and
 * VTM_ERR_INVALID for mixed devices or precisions, VTM_ERR_STATE for a member not set up.
 */
vtm_status vtm_batch_solve(vtm_handle *hs, int32_t count, const double *const *b, int32_t nrhs, const int64_t *ldb,
                           double tol, double *const *x, const int64_t *ldx, int32_t *const *iters,
                           double *const *relres);

/*
 * Run exactly nsweeps FP64-or-FP32 sweeps (handle precision, no refinement)
 * from the current waves, then write the merged potentials of the last sweep
 * to x.  The waves persist across calls (checkpoint/resume with
 * vtm_get_waves / vtm_set_waves).  b, x as in vtm_solve.
 */
vtm_status vtm_run_sweeps(vtm_handle h, const double *b, int32_t nrhs, int64_t ldb, int64_t nsweeps, double *x,
                          int64_t ldx);

/*
 * Autotuner of the sweep launch: times a few sweeps of every candidate
 * (right-hand sides per workgroup R in {1,2,4,8} up to nrhs, workgroup size in
 * {128, 256, 512}) on the current factors with HIP events and keeps the
 * fastest for solves with nrhs right-hand sides; also tries both forward
 * substitution variants and, when the port Green's functions exist, the
 * port-reduced sweep.  chosen[4] = {R, threads, variant, mode} (may be NULL).  The waves are reset.  Requires vtm_setup.
 */
vtm_status vtm_autotune(vtm_handle h, int32_t nrhs, int32_t *chosen);

/* Zero the waves (the state of Example 5.1 before its first iteration). */
vtm_status vtm_reset_waves(vtm_handle h);
/* Incoming waves a_p = u_twin - Z w_twin of the next sweep, host array [nrhs][nports]. */
vtm_status vtm_get_waves(vtm_handle h, double *a, int32_t nrhs);
vtm_status vtm_set_waves(vtm_handle h, const double *a, int32_t nrhs);

/*
 * Learned impedance (an addition to the paper's impedance matching, Section
 * 7.1): an MLP 13 -> 64 -> 64 -> 1 with ReLU predicts delta = ln(Z a_vv) for
 * every VTL from VTM_NUM_FEATURES scale-free features (twelve of its two ends,
 * and the number of subgraphs of its system as the global scale); setup
 * with VTM_Z_LEARNED uses Z = exp(clamp(delta, ln 1/4, ln 256)) / a_vv.
 * Inference and training run on the matrix cores with BF16 operands and FP32
 * accumulation.  Parameter blob (float, VTM_ZMODEL_PARAMS):
 *   mu[13], sigma[13] (input standardisation), W1[64][13], b1[64],
 *   W2[64][64], b2[64], w3[64], b3.
 */
#define VTM_NUM_FEATURES 13
#define VTM_ZMODEL_PARAMS 5147
#define VTM_ZMODEL_TRAIN 5121

/* Features of every VTL (host array [nvtl][VTM_NUM_FEATURES]); works on host-only handles. */
vtm_status vtm_zfeatures(vtm_handle h, float *out);
/* Load model parameters: weights points to bytes = VTM_ZMODEL_PARAMS * 4 bytes (host, copied), the
 * float blob above; another size or a non-finite value gives VTM_ERR_INVALID.  Enables VTM_Z_LEARNED. */
vtm_status vtm_zmodel_load(vtm_handle h, const void *weights, size_t bytes);
/* Impedance per VTL used by the last vtm_setup (host array [nvtl]). */
vtm_status vtm_get_z(vtm_handle h, double *z);

/*
 * Trainer of the impedance model: mean squared error on (features, label)
 * rows held in device memory; minibatch gradients from the same BF16 kernels,
 * Adam (beta 0.9 / 0.999, eps 1e-8) on FP32 master weights.
 */
typedef struct vtm_trainer_ctx *vtm_trainer;
vtm_status vtm_trainer_create(int32_t device, const float *params, vtm_trainer *out);
vtm_status vtm_trainer_destroy(vtm_trainer t);
/* Copy n rows of features [n][VTM_NUM_FEATURES] and labels [n] (host) to the device. */
vtm_status vtm_trainer_set_data(vtm_trainer t, const float *feats, const float *labels, int64_t n);
/* Gradient (host [VTM_ZMODEL_TRAIN], parameter layout without mu/sigma) and loss of rows [row0, row0+nrows). */
vtm_status vtm_trainer_grad(vtm_trainer t, int64_t row0, int64_t nrows, float *grad, float *loss);
/* One epoch: splitmix64-seeded shuffle, minibatches of `batch` rows, one Adam step each; mean loss out. */
vtm_status vtm_trainer_epoch(vtm_trainer t, int64_t batch, float lr, uint64_t seed, float *loss);
/* Model output for n feature rows (host in, host out). */
vtm_status vtm_trainer_predict(vtm_trainer t, const float *feats, int64_t n, float *out);
vtm_status vtm_trainer_get_params(vtm_trainer t, float *params);

/* Statistics of the last setup / solve. */
vtm_status vtm_get_stats(vtm_handle h, vtm_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* VTM_H */
