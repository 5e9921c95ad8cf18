// HIP kernels of libvtm for gfx950 (CDNA4, 64-wide wavefronts).
//
//  k_factor   one workgroup per subgraph: multifrontal Cholesky of the
//             port-augmented matrix K_k of eq. (5.8), level by level; the
//             diagonal block of every supernode is stored inverted so that the
//             sweep has no long sequential chains.  Optionally also the port
//             Green's functions G_k used by the port-reduced sweep (k_schur).
//  k_sweep    one workgroup per (subgraph, group of right-hand sides): one VTM
//             sweep (Table 1 steps 3-5).  Gathers the incoming waves from the
//             twins' outgoing waves of the previous sweep (the delay of (5.6)),
//             forms the right side of (5.8), runs the level-synchronous forward
//             and backward substitutions in LDS and writes the outgoing waves
//             o_p = u_p - Z w_p = 2 u_p - a_p.
//  k_split / k_merge / k_residual: source split b_v/|S(v)|, merged potentials
//             (mean over the children) and the FP64 relative residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "kernels.hpp"

namespace vtm {

namespace {

constexpr int kThreads = 256;
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kWriteX = 1, kNoWaves = 2, kZeroWaves = 4, kWriteY = 8;

__global__ void k_invz(const double *__restrict__ z, const int32_t *__restrict__ port_vtl, double *__restrict__ i64,
                       float *__restrict__ i32, int64_t np) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    double v = 1.0 / z[port_vtl[p]];
    i64[p] = v;
    i32[p] = (float)v;
}

__global__ void k_to_f32(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}

// ---------------------------------------------------------------- factorisation
//
// One workgroup per subgraph walks the assembly tree level by level.  A level whose fronts are
// small is spread over the waves (one supernode per wave at a time, wave-level synchronisation
// only); otherwise the whole workgroup takes its supernodes one after the other.
//
// Fronts that fit in LDS (factor_front): the front F of order f = nc + m is assembled (local
// entries with the port diagonal Z^{-1}, then the children's update matrices) and eliminated by
// nc rank-1 steps that produce everything the sweep and the parent need at once.  With B the
// f x nc right side [I; 0] carried along (forward substitution with the front's unit lower factor),
// step k takes d = sqrt(F[k][k]), scales column k by 1/d and applies the rank-1 update to every
// column c > k over all rows; B[c][i] lives at F[i][c] (i < c, the strictly upper part, which the
// symmetric matrix does not use) and row k of it is reset when k becomes the pivot.  After nc
// steps
//   F[j][i], j <= i < nc   Linv = L11^{-1} (its diagonal 1/d kept beside the front),
//   F[j][nc + q]           -W = -L21 L11^{-1},
//   F[nc + a][nc + b]      the update matrix F22 - L21 L21^T (lower triangle).
// Port Green's functions: with E the unit columns of the port vertices, Y = L^{-1} E and
// G_k = E^T K_k^{-1} E = Y^T Y.  Column j of Y is non-zero only on the supernodes above the one
// holding port j, so s carries just the w_s ports below it (a contiguous range, see DevGreen).  Its
// port front T_s ((nc + m) x w_s, workspace) holds the unit entries of its own ports and what the
// children pushed; [Y_s; U_s] = [Linv; -W] T_s[:nc] + [0; T_s[nc:]] is one product on the FP64
// matrix cores, U_s goes into the parent's port front (siblings own disjoint columns: plain
// stores) and G[ports of s, ports of s] += Y_s^T Y_s (matrix cores; atomic adds that never meet
// another add to the same entry inside one level, so the sums keep their order).
//
// Fronts too large for LDS (factor_node) keep the front in the workspace and run the same
// algebra step by step: Cholesky, Linv, L21, outputs, update (matrix cores), Green's functions.
constexpr int kWaveChol = 48;
constexpr int kPreA = 4, kPreU = 8;  // assembly entries per thread loaded before the first LDS store
constexpr int kTile = 5;             // register tile of the front per thread (rows x columns)

// LDS doubles after the front for the pivot column(s): two padded buffers and spare slots for the
// register elimination, or 2 f for the LDS one (BLK: the team is the workgroup of 256 threads).
__host__ __device__ constexpr int pivot_len(int f, bool blk) {
    return 2 * (blk ? 16 : 8) * kTile + (blk ? 16 : 8) > 2 * f ? 2 * (blk ? 16 : 8) * kTile + (blk ? 16 : 8) : 2 * f;
}
constexpr int kFactorLds = 5056;     // doubles of LDS per workgroup for the fronts (four workgroups per CU)

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// 1 / sqrt(d) for a positive finite d: the hardware estimate (relative error about 2^-23) and three
// Newton steps y <- y (3 - d y^2) / 2, each of which squares the relative error (to rounding level
// after the third); a short dependent chain, unlike a correctly rounded square root and division.
__device__ inline double rsqrt_newton(double d) {
    const double h = 0.5 * d;
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 3; ++it) y = y * fma(-h * y, y, 1.5);
    return y;
}

template <bool BLK>
__device__ inline void team_sync() {
    if (BLK) __syncthreads();
    else wave_sync();
}

// Lower-triangle entry (ta, tb <= ta) of number it in row-major triangular order.
__device__ inline void tri_tile(int it, int &ta, int &tb) {
    ta = (int)((sqrtf(8.0f * (float)it + 1.0f) - 1.0f) * 0.5f);
    while (ta * (ta + 1) / 2 > it) --ta;
    while ((ta + 1) * (ta + 2) / 2 <= it) ++ta;
    tb = it - ta * (ta + 1) / 2;
}

// Cover of a rows x cols rectangle by a team of n threads (n a power of two): the low bits of the
// rank pick the column (stride cw), the high bits the first row (stride rs); no integer division.
struct Cover {
    int c, cw, r0, rs;
};
__device__ inline Cover cover(int cols, int r, int n) {
    int cw = cols <= 1 ? 1 : 1 << (32 - __clz(cols - 1));
    if (cw > n) cw = n;
    const int lw = __ffs(cw) - 1;
    return Cover{r & (cw - 1), cw, r >> lw, n >> lw};
}

// 16 x 16 tile (ta, tb) of P^T P for P (K x n) read through ld(t, col): v_mfma_f64_16x16x4, where
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 j + l / 16][l % 16].  The
// operands of four k-steps are loaded before the first product, so that loads from global memory
// are in flight together.
template <typename LD>
__device__ inline f64x4 gram_tile(int ta, int tb, int K, int n, int lane, LD ld) {
    const int ra = 16 * ta + (lane & 15), rb = 16 * tb + (lane & 15), kr = lane >> 4;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int t0 = 0; t0 < K; t0 += 16) {
        double av[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = t0 + 4 * q + kr;
            av[q] = (t < K && ra < n) ? ld(t, ra) : 0.0;
            bv[q] = (t < K && rb < n) ? ld(t, rb) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (t0 + 4 * q < K) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
    }
    return acc;
}

// Position of G[i][j] in the packed symmetric layout of the port-reduced sweep (lower block
// triangle of 16 x 16 blocks, block column by block column, each block row-major), or -1 for an
// entry of the strictly upper block triangle (not stored).
// Position of entry (i, j) in a 16 x 16 block of G_k: the four column quads one after another, each
// row by row (entry (i, j) at 64 (j / 4) + 4 i + j % 4).  Lane 16 q + m of a wave then reads
// B[m][4 q .. 4 q + 4) as one contiguous 16-byte word, and a wave reads a block in address order.
__device__ inline int gblk_pos(int i, int j) { return 64 * (j >> 2) + 4 * i + (j & 3); }

__device__ inline int64_t gpack_index(int nb, int i, int j) {
    const int I = i >> 4, J = j >> 4;
    if (I < J) return -1;
    return ((int64_t)J * nb - (int64_t)J * (J - 1) / 2 + (I - J)) * 256 + gblk_pos(i & 15, j & 15);
}

// Stored factor of a supernode with nc columns and f = nc + m rows: V = [Linv; W] (Linv = L11^{-1}
// lower triangular, W = L21 L11^{-1}), only its lower trapezoid, column by column: column j holds rows
// j .. f - 1 contiguously (Linv rows j .. nc - 1, then the m rows of W), so V[i][j], i >= j, sits at
// vpos(f, i, j).  nc (nc + 1) / 2 + m nc values.  The forward substitution reads each column once as
// an axpy (lanes over rows), the backward one each column once as a dot product (lanes over the
// column's rows); both reads are coalesced.
__host__ __device__ inline int vcol(int f, int j) { return j * f - j * (j - 1) / 2; }
__host__ __device__ inline int vpos(int f, int i, int j) { return vcol(f, j) + (i - j); }

struct FactorArgs {
    const double *A;       // assembly values of the subgraph (scatter order)
    double *V;             // factor values of the subgraph (FP64), or nullptr
    float *V32;            // the same in FP32, or nullptr
    double *W;             // update-matrix workspace of the subgraph
    const double *dplus;   // port diagonal per factor position
    const int32_t *sn_c0, *sn_nc, *sn_m, *sn_val, *sn_uoff, *sn_ridx;
    const int32_t *ch_ptr, *ch_idx, *sc_ptr, *sc_dst;
    const uint16_t *rel;
    // port Green's functions (gpl == nullptr: not computed)
    const int4 *gpl;
    double *gws;
    float *gws32;  // FP32 copy of the Y blocks (at y32_pos), or nullptr
    const uint16_t *perm;
    double *Gk;
    int nb;  // 16 x 16 blocks per row of the packed G_k
};

// Position of Y_s[row][a] in the FP32 copy of the Y blocks: column-major from the start of the
// supernode's region of the Green workspace (which holds (2 nc + m) w >= nc w entries), so that the
// threads of a test solve, one per row, read consecutive entries for every port column a.
__host__ __device__ inline int64_t y32_pos(int64_t region, int nc, int row, int a) {
    return region + (int64_t)a * nc + row;
}

// G[ports a, b of s] += acc for the lower part of tile (ta, tb) of Y_s^T Y_s; port(x) is the port
// number of column x of s.
template <typename PORT>
__device__ inline void green_add(const FactorArgs &X, int w, int ta, int tb, int lane, const f64x4 &acc, PORT port) {
    const int b = 16 * tb + (lane & 15), kr = lane >> 4;
    const int jb = port(b);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int a = 16 * ta + 4 * j + kr;
        const int ja = port(a);
        if (a < w && b < w && b <= a) {
            const int64_t e1 = gpack_index(X.nb, ja, jb), e2 = gpack_index(X.nb, jb, ja);
            if (e1 >= 0) atomicAdd(X.Gk + e1, acc[j]);
            if (a != b && e2 >= 0) atomicAdd(X.Gk + e2, acc[j]);
        }
    }
}

// Elimination of a front held in registers: the team is a G x G grid (G = 8 for a wave, 16 for the
// workgroup) and thread (lr, lc) keeps the entries (lr + G a, lc + G b), a, b < KT, of F.  Step k reads
// only the pivot column, published in one of two LDS buffers (pk and pk + kPad, each kPad = G kTile
// long, so that rows past the front need no guard; G spare slots follow) by the threads owning it; a
// step costs one barrier.  Column k is final after step k: its rows <= k (row k of B and the diagonal 1/d of Linv)
// go straight to the front, its other rows are never read again.  Row k restarts from zero as row
// k of B.  Columns < k keep being updated in registers but are never read
// again; columns >= nc go back to the front at the end.
template <int KT, bool BLK>
__device__ __forceinline__ void elim_regs(double *F, double *pk, int f, int nc, int r, int s, int *sbad) {
    constexpr int G = BLK ? 16 : 8, kPad = G * kTile;
    const int lr = r / G, lc = r & (G - 1);
    double v[KT][KT];
#pragma unroll
    for (int a = 0; a < KT; ++a)
#pragma unroll
        for (int b = 0; b < KT; ++b) {
            const int i = lr + G * a, c = lc + G * b;
            v[a][b] = i < f && c < f ? F[i * f + c] : 0.0;
        }
    if (lc == 0)
#pragma unroll
        for (int a = 0; a < KT; ++a) pk[lr + G * a] = v[a][0];
    team_sync<BLK>();
    for (int k = 0; k < nc; ++k) {
        const double *cb = pk + (k & 1) * kPad;
        double *cn = pk + (~k & 1) * kPad;
        // every read of the step at once (the buffer is kPad long: no guards), so the step waits for
        // LDS once
        double d = cb[k], ci[KT], cc[KT];
#pragma unroll
        for (int a = 0; a < KT; ++a) ci[a] = cb[lr + G * a];
#pragma unroll
        for (int b = 0; b < KT; ++b) cc[b] = cb[lc + G * b];
        if (!(d > 0.0) || !isfinite(d)) {
            if (r == 0) atomicMin(sbad, s + 1);
            d = 1.0;
        }
        const double rd = rsqrt_newton(d);
        double pi[KT];
#pragma unroll
        for (int a = 0; a < KT; ++a) pi[a] = lr + G * a == k ? rd : ci[a] * rd;
        if (lc == 0)  // the finished column: rows <= k into the front (row k of B, diagonal of Linv)
#pragma unroll
            for (int a = 0; a < KT; ++a) {
                const int i = lr + G * a;
                double *dst = i < f ? F + i * f + k : pk + 2 * kPad + lr;  // rows past the front: spare slots
                *dst = pi[a];  // rows k < i < f are entries of L that nothing reads
            }
        if (lr == (k & (G - 1))) {  // row k restarts as row k of B
            const int aa = k / G;
#pragma unroll
            for (int a = 0; a < KT; ++a)
                if (a == aa)
#pragma unroll
                    for (int b = 0; b < KT; ++b) v[a][b] = 0.0;
        }
#pragma unroll
        for (int b = 0; b < KT; ++b) {
            const double pc = cc[b] * rd;
#pragma unroll
            for (int a = 0; a < KT; ++a) v[a][b] = fma(-pi[a], pc, v[a][b]);
        }
        if (k + 1 < nc && lc == ((k + 1) & (G - 1))) {  // publish column k + 1
            const int bb = (k + 1) / G;
#pragma unroll
            for (int b = 0; b < KT; ++b)
                if (b == bb)
#pragma unroll
                    for (int a = 0; a < KT; ++a) cn[lr + G * a] = v[a][b];
        }
        team_sync<BLK>();
    }
#pragma unroll
    for (int a = 0; a < KT; ++a)
#pragma unroll
        for (int b = 0; b < KT; ++b) {
            const int i = lr + G * a, c = lc + G * b;
            if (i < f && c < f && c >= nc) F[i * f + c] = v[a][b];
        }
    team_sync<BLK>();
}

// Supernode s by a team of n threads (rank r; wv / nw: its wave in the team and the team's
// waves; n = 64 for a wave, 256 for the workgroup) in the LDS region F of cap doubles: the front
// (f x f), the pivot-column buffers (pivot_len) and, when room is left, Y_s (nc x w_s).
template <bool BLK>
__device__ __forceinline__ void factor_front(const FactorArgs &X, int s, double *F, int cap, int r, int n, int wv, int nw,
                             int *sbad) {
    s = __builtin_amdgcn_readfirstlane(s);  // the same supernode in every lane of the wave
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane), "+v"(r));  // lane-derived values are recomputed per supernode, not kept live
    const int c0 = X.sn_c0[s], nc = X.sn_nc[s], m = X.sn_m[s], f = nc + m;
    double *pk = F + f * f;
    const int sc0 = X.sc_ptr[s], nsc = X.sc_ptr[s + 1] - sc0;
    const int ch0 = X.ch_ptr[s], nch = X.ch_ptr[s + 1] - ch0;
    // 1. assembly.  The loads of the common case (this thread's first kPreA local entries, with the
    //    port diagonal on the first nc, which are the diagonals of the own columns; its first kPreU
    //    entries of the first two children's packed update matrices) are all issued before the
    //    front is cleared, so the supernode waits for memory once.
    double av[kPreA];
    int ap[kPreA];
#pragma unroll
    for (int q = 0; q < kPreA; ++q) {
        const int e = r + q * n;
        ap[q] = -1;
        av[q] = 0.0;
        if (e < nsc) {
            ap[q] = X.sc_dst[sc0 + e];
            av[q] = X.A[sc0 + e] + (e < nc ? X.dplus[c0 + e] : 0.0);
        }
    }
    double uv[2][kPreU];
    int up[2][kPreU];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int mc = 0;
        const double *U = nullptr;
        const uint16_t *rc = nullptr;
        if (h < nch) {
            const int c = X.ch_idx[ch0 + h];
            mc = X.sn_m[c];
            U = X.W + X.sn_uoff[c];
            rc = X.rel + X.sn_ridx[c];
        }
        const int nt = mc * (mc + 1) / 2;
#pragma unroll
        for (int q = 0; q < kPreU; ++q) {
            const int t = r + q * n;
            up[h][q] = -1;
            uv[h][q] = 0.0;
            if (t < nt) {
                int a, b;
                tri_tile(t, a, b);
                up[h][q] = rc[a] * f + rc[b];
                uv[h][q] = U[t];
            }
        }
    }
    for (int i = r; i < f * f; i += n) F[i] = 0.0;
    team_sync<BLK>();
#pragma unroll
    for (int q = 0; q < kPreA; ++q)
        if (ap[q] >= 0) F[ap[q]] = av[q];
    for (int e = r + kPreA * n; e < nsc; e += n) F[X.sc_dst[sc0 + e]] = X.A[sc0 + e] + (e < nc ? X.dplus[c0 + e] : 0.0);
    for (int h = 0; h < nch; ++h) {  // children one after the other: their rows overlap
        team_sync<BLK>();
        const int c = X.ch_idx[ch0 + h], mc = X.sn_m[c], nt = mc * (mc + 1) / 2;
        const double *U = X.W + X.sn_uoff[c];
        const uint16_t *rc = X.rel + X.sn_ridx[c];
        int t = r;
        if (h == 0 || h == 1) {
#pragma unroll
            for (int q = 0; q < kPreU; ++q) {
                const int p = h == 0 ? up[0][q] : up[1][q];
                if (p >= 0) F[p] += h == 0 ? uv[0][q] : uv[1][q];
            }
            t = r + kPreU * n;
        }
        for (; t < nt; t += n) {
            int a, b;
            tri_tile(t, a, b);
            F[rc[a] * f + rc[b]] += U[t];
        }
    }
    team_sync<BLK>();
    // 2. elimination: nc rank-1 steps (see the section comment)
    constexpr int G = BLK ? 16 : 8;  // the team as a G x G grid of threads
    if (f <= 3 * G) {
        elim_regs<3, BLK>(F, pk, f, nc, r, s, sbad);
    } else if (f <= kTile * G) {
        elim_regs<kTile, BLK>(F, pk, f, nc, r, s, sbad);
    } else {
        for (int k = 0; k < nc; ++k) {
            double d = F[k * f + k];
            if (!(d > 0.0) || !isfinite(d)) {
                if (r == 0) atomicMin(sbad, s + 1);
                d = 1.0;
            }
            const double rd = rsqrt_newton(d);
            for (int i = r; i < f; i += n) {
                const double p = i == k ? rd : F[i * f + k] * rd;
                pk[i] = p;
                if (i < k) F[i * f + k] = p;  // row k of B, final
            }
            team_sync<BLK>();
            if (r == 0) F[k * f + k] = rd;  // diagonal of Linv
            const int ncol = f - k - 1;
            if (ncol > 0) {
                const Cover cv = cover(ncol, r, n);
                for (int cc = cv.c; cc < ncol; cc += cv.cw) {
                    const int c = k + 1 + cc;
                    const double pc = pk[c];
                    for (int i = cv.r0; i < f; i += cv.rs) {
                        double *q = F + i * f + c;
                        *q = (i == k ? 0.0 : *q) - pk[i] * pc;
                    }
                }
            }
            team_sync<BLK>();
        }
    }
    // 3. outputs: [Linv; W] (f x nc, lower trapezoid, packed by columns: see vpos), the update matrix
    //    (packed lower triangle)
    {
        double *Vs = X.V ? X.V + X.sn_val[s] : nullptr;
        float *Vs32 = X.V32 ? X.V32 + X.sn_val[s] : nullptr;
        const Cover cv = cover(nc, r, n);
        for (int j = cv.c; j < nc; j += cv.cw)
            for (int i = cv.r0; i < f; i += cv.rs) {
                if (i < j) continue;
                const double v = i < nc ? F[j * f + i] : -F[j * f + i];
                if (Vs) Vs[vpos(f, i, j)] = v;
                if (Vs32) Vs32[vpos(f, i, j)] = (float)v;
            }
    }
    if (m > 0) {
        double *Us = X.W + X.sn_uoff[s];
        const Cover cv = cover(m, r, n);
        for (int b = cv.c; b < m; b += cv.cw)
            for (int a = cv.r0; a < m; a += cv.rs)
                if (b <= a) Us[a * (a + 1) / 2 + b] = F[(nc + a) * f + nc + b];
    }
    // 4. port Green's functions through s
    if (X.gpl) {
        const int4 e = X.gpl[s];
        const int w = (int)((uint32_t)e.y >> 16), pc0 = e.y & 0xFFFF;
        if (w > 0) {
            double *T = X.gws + e.x;
            double *Yg = X.gws + e.x + (int64_t)f * w;
            const int pw = (int)((uint32_t)e.w >> 16), ppc0 = e.w & 0xFFFF;
            const uint16_t *rs_ = X.rel + X.sn_ridx[s];
            // the parent rows of the update rows and the port numbers of s, two per lane (read through
            // lane shuffles below, so that no global load sits behind this supernode's stores)
            const bool rsh = m <= 128, psh = w <= 128;
            int rv0 = 0, rv1 = 0, pv0 = 0, pv1 = 0;
            if (rsh) {
                rv0 = lane < m ? rs_[lane] : 0;
                rv1 = lane + 64 < m ? rs_[lane + 64] : 0;
            }
            if (psh) {
                pv0 = lane < w ? X.perm[pc0 + lane] : 0;
                pv1 = lane + 64 < w ? X.perm[pc0 + lane + 64] : 0;
            }
            const auto prow_of = [&](int q) {  // parent row of update row q (all lanes call it)
                if (!rsh) return q >= 0 && q < m ? (int)rs_[q] : 0;
                const int x0 = __shfl(rv0, q & 63), x1 = __shfl(rv1, q & 63);
                return q < 64 ? x0 : x1;
            };
            const auto port_of = [&](int x) {  // port number of column x of s (all lanes call it)
                if (!psh) return x < w ? (int)X.perm[pc0 + x] : 0;
                const int x0 = __shfl(pv0, x & 63), x1 = __shfl(pv1, x & 63);
                return x < 64 ? x0 : x1;
            };
            // LDS after the product's operand rows F[:nc] (the rest of the front is consumed): the port
            // front T (f x w) and Y (nc x w) when both fit; else Y alone after the pivot buffers
            const int offT = nc * f, offY = offT + f * w;
            const bool staged = offY + nc * w <= cap;
            double *Ts = staged ? F + offT : nullptr;
            double *Yl = staged ? F + offY
                                : (f * f + pivot_len(f, BLK) + nc * w <= cap ? pk + pivot_len(f, BLK) : nullptr);
            if (staged) {
                team_sync<BLK>();  // the outputs have read the front
                for (int i0 = r; i0 < f * w; i0 += 16 * n) {
                    double t[16];
#pragma unroll
                    for (int q = 0; q < 16; ++q) t[q] = i0 + q * n < f * w ? T[i0 + q * n] : 0.0;
#pragma unroll
                    for (int q = 0; q < 16; ++q)
                        if (i0 + q * n < f * w) {
                            Ts[i0 + q * n] = t[q];
                            T[i0 + q * n] = 0.0;  // the port front is left zero for the next factorisation
                        }
                }
                team_sync<BLK>();
            }
            const double *Tp = staged ? Ts : T;
            const int tr = (f + 15) >> 4, tcn = (w + 15) >> 4, kr = lane >> 4, l16 = lane & 15;
            // [Y; U] = [Linv; -W] T[:nc] + [0; T[nc:]], 16 x 16 tiles over (rows of the front, ports)
            for (int it = wv; it < tr * tcn; it += nw) {
                const int ti = it / tcn, tj = it - ti * tcn;
                const int i = 16 * ti + l16, a = 16 * tj + l16;
                double tadd[4];
                int prow[4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int row = 16 * ti + 4 * jj + kr;
                    const bool low = row >= nc && row < f;
                    tadd[jj] = low && a < w ? Tp[row * w + a] : 0.0;
                    prow[jj] = prow_of(row - nc);
                }
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
                for (int k0 = 0; k0 < nc; k0 += 16) {
                    double bv[4], lv[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int j = k0 + 4 * q + kr;
                        bv[q] = j < nc && a < w ? Tp[j * w + a] : 0.0;
                        lv[q] = j < nc && i < f && j <= i ? F[j * f + i] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (k0 + 4 * q < nc) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(lv[q], bv[q], acc, 0, 0, 0);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int row = 16 * ti + 4 * jj + kr;
                    if (row < f && a < w) {
                        const double v = acc[jj] + tadd[jj];
                        if (row < nc) {
                            Yg[row * w + a] = v;
                            if (Yl) Yl[row * w + a] = v;
                            if (X.gws32) X.gws32[y32_pos(e.x, nc, row, a)] = (float)v;
                        } else {
                            X.gws[e.z + (int64_t)prow[jj] * pw + a + (pc0 - ppc0)] = v;
                        }
                    }
                }
            }
            team_sync<BLK>();
            if (!staged)  // the port front is left zero for the next factorisation
                for (int i = r; i < f * w; i += n) T[i] = 0.0;
            if (X.Gk && !Yl && nc * w <= cap) {  // the front is consumed: Y_s over it, so the Gram products read LDS
                for (int i0 = r; i0 < nc * w; i0 += 8 * n) {
                    double t[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) t[q] = i0 + q * n < nc * w ? Yg[i0 + q * n] : 0.0;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (i0 + q * n < nc * w) F[i0 + q * n] = t[q];
                }
                Yl = F;
                team_sync<BLK>();
            }
            for (int it = wv; X.Gk && it < tcn * (tcn + 1) / 2; it += nw) {  // G += Y^T Y
                int ta, tb;
                tri_tile(it, ta, tb);
                const f64x4 acc = Yl ? gram_tile(ta, tb, nc, w, lane, [&](int t, int c) { return Yl[t * w + c]; })
                                     : gram_tile(ta, tb, nc, w, lane, [&](int t, int c) { return Yg[t * w + c]; });
                green_add(X, w, ta, tb, lane, acc, port_of);
            }
        }
    }
    team_sync<BLK>();
}

// Supernode s by the workgroup with its front F in the workspace (fronts too large for LDS).
__device__ __forceinline__ void factor_node(const FactorArgs &X, int s, double *F, int r, int n, int wv, int nw, int *sbad) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane), "+v"(r));  // lane-derived values are recomputed per supernode, not kept live
    const int c0 = X.sn_c0[s], nc = X.sn_nc[s], m = X.sn_m[s], f = nc + m;
    // 1. assembly
    for (int i = r; i < f * f; i += n) F[i] = 0.0;
    __syncthreads();
    for (int e = X.sc_ptr[s] + r; e < X.sc_ptr[s + 1]; e += n) F[X.sc_dst[e]] = X.A[e];
    __syncthreads();
    for (int j = r; j < nc; j += n) F[j * f + j] += X.dplus[c0 + j];
    for (int q = X.ch_ptr[s]; q < X.ch_ptr[s + 1]; ++q) {  // children one at a time (they share rows)
        __syncthreads();
        const int c = X.ch_idx[q], mc = X.sn_m[c];
        const double *U = X.W + X.sn_uoff[c];
        const uint16_t *rc = X.rel + X.sn_ridx[c];
        for (int t = r; t < mc * (mc + 1) / 2; t += n) {
            int a, b;
            tri_tile(t, a, b);
            F[rc[a] * f + rc[b]] += U[t];
        }
    }
    __syncthreads();
    // 2. Cholesky of the diagonal block (right-looking; one wave when nc <= kWaveChol)
    if (nc <= kWaveChol) {
        if (wv == 0) {
            for (int kk = 0; kk < nc; ++kk) {
                double d = F[kk * f + kk];
                if (!(d > 0.0) || !isfinite(d)) {
                    if (lane == 0) atomicMin(sbad, s + 1);
                    d = 1.0;
                }
                const double sd = sqrt(d), rs = 1.0 / sd;
                wave_sync();
                for (int i = kk + 1 + lane; i < nc; i += 64) F[i * f + kk] *= rs;
                if (lane == 0) F[kk * f + kk] = sd;
                wave_sync();
                const int T = nc - kk - 1;
                for (int idx = lane; idx < T * T; idx += 64) {
                    const int i = kk + 1 + idx / T, j = kk + 1 + idx % T;
                    if (j <= i) F[i * f + j] -= F[i * f + kk] * F[j * f + kk];
                }
                wave_sync();
            }
        }
    } else {
        for (int kk = 0; kk < nc; ++kk) {
            double d = F[kk * f + kk];
            if (!(d > 0.0) || !isfinite(d)) {
                if (r == 0) atomicMin(sbad, s + 1);
                d = 1.0;
            }
            const double sd = sqrt(d), rs = 1.0 / sd;
            __syncthreads();
            for (int i = kk + 1 + r; i < nc; i += n) F[i * f + kk] *= rs;
            if (r == 0) F[kk * f + kk] = sd;
            __syncthreads();
            const int T = nc - kk - 1;
            for (int idx = r; idx < T * T; idx += n) {
                const int i = kk + 1 + idx / T, j = kk + 1 + idx % T;
                if (j <= i) F[i * f + j] -= F[i * f + kk] * F[j * f + kk];
            }
            __syncthreads();
        }
    }
    __syncthreads();
    // 3. Linv[i][j] = -(sum_{j <= t < i} L[i][t] Linv[t][j]) / L[i][i], stored at F[j][i]
    for (int j = r; j < nc; j += n) {
        const double djj = 1.0 / F[j * f + j];
        for (int i = j + 1; i < nc; ++i) {
            double acc = F[i * f + j] * djj;
            for (int t = j + 1; t < i; ++t) acc += F[i * f + t] * F[j * f + t];
            F[j * f + i] = -acc / F[i * f + i];
        }
    }
    __syncthreads();
    // 4. L21[q][t] = sum_{u <= t} F21[q][u] Linv[t][u], stored at F[t][nc + q]
    for (int idx = r; idx < m * nc; idx += n) {
        const int q = idx / nc, t = idx - q * nc;
        const double *row = F + (nc + q) * f;
        double acc = row[t] / F[t * f + t];
        for (int u = 0; u < t; ++u) acc += row[u] * F[u * f + t];
        F[t * f + nc + q] = acc;
    }
    __syncthreads();
    // 5. outputs
    double *Vs = X.V ? X.V + X.sn_val[s] : nullptr;
    float *Vs32 = X.V32 ? X.V32 + X.sn_val[s] : nullptr;
    for (int idx = r; idx < nc * nc; idx += n) {
        const int i = idx / nc, j = idx - i * nc;
        if (j > i) continue;
        const double v = j == i ? 1.0 / F[i * f + i] : F[j * f + i];
        if (Vs) Vs[vpos(f, i, j)] = v;
        if (Vs32) Vs32[vpos(f, i, j)] = (float)v;
    }
    for (int idx = r; idx < m * nc; idx += n) {  // W[q][j] = sum_{t >= j} L21[q][t] Linv[t][j]
        const int q = idx / nc, j = idx - q * nc;
        double acc = F[j * f + nc + q] / F[j * f + j];
        for (int t = j + 1; t < nc; ++t) acc += F[t * f + nc + q] * F[j * f + t];
        if (Vs) Vs[vpos(f, nc + q, j)] = acc;
        if (Vs32) Vs32[vpos(f, nc + q, j)] = (float)acc;
    }
    double *Us = X.W + X.sn_uoff[s];
    const int tm = (m + 15) >> 4, kr = lane >> 4;
    for (int it = wv; it < tm * (tm + 1) / 2; it += nw) {  // update = F22 - L21 L21^T, packed lower
        int ta, tb;
        tri_tile(it, ta, tb);
        const f64x4 acc = gram_tile(ta, tb, nc, m, lane, [&](int t, int a) { return F[t * f + nc + a]; });
        const int b = 16 * tb + (lane & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = 16 * ta + 4 * j + kr;
            if (a < m && b < m && b <= a) Us[a * (a + 1) / 2 + b] = F[(nc + a) * f + nc + b] - acc[j];
        }
    }
    // 6. port Green's functions through s
    if (X.gpl) {
        const int4 e = X.gpl[s];
        const int w = (int)((uint32_t)e.y >> 16), pc0 = e.y & 0xFFFF;
        if (w > 0) {
            double *T = X.gws + e.x;
            double *Y = X.gws + e.x + (int64_t)f * w;
            const int pw = (int)((uint32_t)e.w >> 16), ppc0 = e.w & 0xFFFF;
            const uint16_t *rs_ = X.rel + X.sn_ridx[s];
            for (int idx = r; idx < nc * w; idx += n) {  // Y = Linv T
                const int i = idx / w, a = idx - i * w;
                double acc = T[i * w + a] / F[i * f + i];
                for (int t = 0; t < i; ++t) acc += F[t * f + i] * T[t * w + a];
                Y[idx] = acc;
                if (X.gws32) X.gws32[y32_pos(e.x, nc, i, a)] = (float)acc;
            }
            __syncthreads();
            for (int idx = r; idx < m * w; idx += n) {  // T[nc:] - L21 Y into the parent's port front
                const int q = idx / w, a = idx - q * w;
                double acc = T[(nc + q) * w + a];
                for (int t = 0; t < nc; ++t) acc -= F[t * f + nc + q] * Y[t * w + a];
                X.gws[e.z + (int64_t)rs_[q] * pw + a + (pc0 - ppc0)] = acc;
            }
            __syncthreads();
            for (int i = r; i < f * w; i += n) T[i] = 0.0;  // the port front is left zero for the next factorisation
            const int tw = (w + 15) >> 4;
            for (int it = wv; X.Gk && it < tw * (tw + 1) / 2; it += nw) {  // G += Y^T Y
                int ta, tb;
                tri_tile(it, ta, tb);
                const f64x4 acc = gram_tile(ta, tb, nc, w, lane, [&](int t, int a) { return Y[t * w + a]; });
                green_add(X, w, ta, tb, lane, acc, [&](int x) { return x < w ? (int)X.perm[pc0 + x] : 0; });
            }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads, 4) void k_factor(DevSym S, DevSub D, const double *__restrict__ aval,
                                                     const double *__restrict__ invz, double *__restrict__ vals,
                                                     float *__restrict__ vals32, double *__restrict__ ws, int lds_doubles,
                                                     int32_t *__restrict__ status, DevGreen Gp,
                                                     const int64_t *__restrict__ goff, double *__restrict__ G) {
    extern __shared__ double sm[];
    __shared__ int sbad;
    const int k = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    const ClassDev C = S.cls[D.cls[k]];
    const int nk = C.nk;
    FactorArgs X;
    X.A = aval + D.aval[k];
    X.V = vals ? vals + D.val[k] : nullptr;
    X.V32 = vals32 ? vals32 + D.val[k] : nullptr;
    X.W = ws + D.ws[k];
    double *dplus = X.W + C.ws_u + (int64_t)C.max_front * C.max_front;
    X.dplus = dplus;
    X.sn_c0 = S.sn_c0 + C.o_sn;
    X.sn_nc = S.sn_nc + C.o_sn;
    X.sn_m = S.sn_m + C.o_sn;
    X.sn_val = S.sn_val + C.o_sn;
    X.sn_uoff = S.sn_uoff + C.o_sn;
    X.sn_ridx = S.sn_ridx + C.o_sn;
    X.ch_ptr = S.ch_ptr + C.o_snp;
    X.ch_idx = S.ch_idx + C.o_chi;
    X.sc_ptr = S.sc_ptr + C.o_snp;
    X.sc_dst = S.sc_dst + C.o_sc;
    X.rel = S.rel + C.o_ridx;
    const int pg0 = D.pg_ptr[k], p = D.pg_ptr[k + 1] - pg0;
    X.gpl = nullptr;
    if (Gp.sn && p > 0) {
        X.gpl = Gp.sn + Gp.base[k];
        X.gws = Gp.ws + Gp.wso[k];
        X.gws32 = Gp.ws32 ? Gp.ws32 + Gp.wso[k] : nullptr;
        X.perm = Gp.perm + pg0;
        X.Gk = G ? G + goff[k] : nullptr;  // nullptr: k_gram forms G_k from the stored Y blocks
        X.nb = (p + 15) >> 4;
        for (int a = tid; a < p; a += nt) X.gws[Gp.idoff[pg0 + a]] = 1.0;
    }
    const int32_t *col_sn = S.col_sn + C.o_col, *lev_c0 = S.lev_c0 + C.o_lev, *lev_maxf = S.lev_maxf + C.o_lev;
    // diagonal additions Z^{-1} of the ports, one thread per port vertex (ports in order)
    for (int i = tid; i < nk; i += nt) dplus[i] = 0.0;
    if (tid == 0) sbad = 0x7FFFFFFF;
    __syncthreads();
    for (int g = D.pg_ptr[k] + tid; g < D.pg_ptr[k + 1]; g += nt) {
        double s = 0.0;
        for (int j = 0; j < D.pg_cnt[g]; ++j) s += invz[D.pg_beg[g] + j];
        dplus[D.pg_pos[g]] = s;
    }
    __syncthreads();
    for (int lv = 0; lv < C.nlev; ++lv) {
        const int s0 = col_sn[lev_c0[lv]], s1 = lv + 1 < C.nlev ? col_sn[lev_c0[lv + 1]] : C.nsn;
        const int mf = lev_maxf[lv], need_w = mf * mf + pivot_len(mf, false), need_b = mf * mf + pivot_len(mf, true);
        const int fit = lds_doubles / need_w, nwa = fit < nw ? fit : nw;
        if (s1 - s0 > 1 && nwa >= 2) {  // one supernode per wave, nwa waves at a time
            const int cap = lds_doubles / nwa;
            if (wv < nwa)
                for (int s = s0 + wv; s < s1; s += nwa) factor_front<false>(X, s, sm + wv * cap, cap, lane, 64, 0, 1, &sbad);
        } else if (need_b <= lds_doubles) {
            for (int s = s0; s < s1; ++s) factor_front<true>(X, s, sm, lds_doubles, tid, nt, wv, nw, &sbad);
        } else {
            for (int s = s0; s < s1; ++s) factor_node(X, s, X.W + C.ws_u, tid, nt, wv, nw, &sbad);
        }
        // every store and atomic add of this level lands before the next level reads or adds
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    if (tid == 0) status[k] = sbad == 0x7FFFFFFF ? 0 : sbad;
}

// G_k = sum over supernodes s of Y_s^T Y_s, one 16 x 16 block of the packed lower block triangle per
// wave, written once (no atomics, no clearing).  The ports below s are the range [lo_s, lo_s + w_s)
// of the plan order, which is also G_k's port order, so block (I, J) gathers the supernodes whose
// range meets both ports 16 I .. 16 I + 15 and 16 J .. 16 J + 15 (the common ancestors of its ports),
// in increasing order, on one chain of v_mfma_f64_16x16x4 (lane l: A[l % 16][l / 16] = Y_s[t][i - lo_s],
// B[l / 16][l % 16] = Y_s[t][j - lo_s], D[4 q + l / 16][l % 16] in acc[q]).  Entries past the last
// port are written as zeros (the padding of the last block).
__global__ __launch_bounds__(256) void k_gram(DevSym S, DevSub D, DevGreen Gp, const int64_t *__restrict__ goff,
                                              double *__restrict__ G) {
    const int k = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int p = D.pg_ptr[k + 1] - D.pg_ptr[k];
    if (p == 0) return;
    const ClassDev C = S.cls[D.cls[k]];
    const int nb = (p + 15) >> 4, ntile = nb * (nb + 1) / 2;
    const int4 *pl = Gp.sn + Gp.base[k];
    const int32_t *sn_nc = S.sn_nc + C.o_sn, *sn_m = S.sn_m + C.o_sn;
    const double *ws = Gp.ws + Gp.wso[k];
    double *Gk = G + goff[k];
    const int l16 = lane & 15, kr = lane >> 4;
    for (int it = blockIdx.y * 4 + wv; it < ntile; it += gridDim.y * 4) {
        int ti, tj;
        tri_tile(it, ti, tj);
        const int i0 = 16 * ti, j0 = 16 * tj;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int s = 0; s < C.nsn; ++s) {
            const int4 e = pl[s];
            const int w = (int)((uint32_t)e.y >> 16), lo = e.y & 0xFFFF;
            if (w == 0 || lo >= i0 + 16 || lo + w <= i0 || lo >= j0 + 16 || lo + w <= j0) continue;
            const int nc = sn_nc[s], f = nc + sn_m[s];
            const double *Y = ws + e.x + (int64_t)f * w;  // Y_s, nc x w row-major
            const int ci = i0 + l16 - lo, cj = j0 + l16 - lo;
            const bool vi = ci >= 0 && ci < w, vj = cj >= 0 && cj < w;
            for (int t0 = 0; t0 < nc; t0 += 16) {
                double av[4], bv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int t = t0 + 4 * q + kr;
                    av[q] = t < nc && vi ? Y[(int64_t)t * w + ci] : 0.0;
                    bv[q] = t < nc && vj ? Y[(int64_t)t * w + cj] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (t0 + 4 * q < nc) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
            }
        }
        const int j = j0 + l16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + 4 * q + kr;
            Gk[gpack_index(nb, i, j)] = i < p && j < p ? acc[q] : 0.0;
        }
    }
}

// ------------------------------------------------------------------------ split
template <typename T>
__global__ void k_split(DevMaps M, int64_t nsplit, const double *__restrict__ b, int32_t nrhs, int32_t S, int32_t R,
                        T *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nsplit) return;
    const int32_t v = M.fvtx[e];
    const double m = (double)M.fmul[e];
    const int ng = (nrhs + R - 1) / R;
    for (int g = 0; g < ng; ++g)
        for (int cc = 0; cc < R; ++cc) {
            const int c = g * R + cc;
            out[((int64_t)g * nsplit + e) * R + cc] = c < nrhs ? (T)(b[(int64_t)v * S + c] / m) : (T)0;
        }
}

// Restart of the listed subgraphs: split of the new right side over their entries, zero waves on
// their ports (for every RHS group).  Entries of subgraph k end where those of k + 1 begin.
template <typename T>
__global__ void k_restart(DevSub D, DevMaps M, int32_t nsub, int64_t nsplit, int64_t nports,
                          const double *__restrict__ b, int32_t nrhs, int32_t S, int32_t R, T *__restrict__ out,
                          T *__restrict__ o) {
    const int k = sub_of_block(D, blockIdx.x);
    const int64_t e0 = D.x[k], e1 = k + 1 < nsub ? D.x[k + 1] : nsplit;
    const int ng = (nrhs + R - 1) / R;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int32_t v = M.fvtx[e];
        const double m = (double)M.fmul[e];
        for (int g = 0; g < ng; ++g)
            for (int cc = 0; cc < R; ++cc) {
                const int c = g * R + cc;
                out[((int64_t)g * nsplit + e) * R + cc] = c < nrhs ? (T)(b[(int64_t)v * S + c] / m) : (T)0;
            }
    }
    const int p0 = D.port_ptr[k], np = D.port_ptr[k + 1] - p0;
    for (int i = threadIdx.x; i < np * R * ng; i += blockDim.x) {
        const int g = i / (np * R), j = i - g * np * R;
        o[((int64_t)g * nports + p0) * R + j] = (T)0;
    }
}

// Lane moves by DPP (quad permutations and row rotations); a double moves as its two halves.
template <int CTRL>
__device__ inline float dpp_mov(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_mov(double v) {
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// Value of lane m ^ X (X = 8, 1, 2 or 4) within each 16-lane DPP row: row_ror:8 for 8, quad
// permutations for 1 and 2, and for 4 a shift left by 4 into banks 0 and 2 plus a shift right by 4
// into banks 1 and 3.
template <int X>
__device__ inline int lane_xor(int v) {
    if constexpr (X == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
    if constexpr (X == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    if constexpr (X == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    if constexpr (X == 4) {
        const int lo = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xF, 0x5, false);
        return __builtin_amdgcn_update_dpp(lo, v, 0x114, 0xF, 0xA, false);
    }
    return v;
}
template <int X>
__device__ inline float lane_xor(float v) {
    return __builtin_bit_cast(float, lane_xor<X>(__builtin_bit_cast(int, v)));
}
template <int X>
__device__ inline double lane_xor(double v) {
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = lane_xor<X>((int)x), hi = lane_xor<X>((int)(x >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum of v over the 16 lanes of each DPP row, left in every lane of the row.
template <typename T>
__device__ inline T row16_sum(T v) {
    v += lane_xor<8>(v);
    v += lane_xor<4>(v);
    v += lane_xor<2>(v);
    v += lane_xor<1>(v);
    return v;
}

// ------------------------------------------------------------------------ sweep
//
// Factor layout per supernode s (nc columns, m off-diagonal rows R_s): Linv_s = L11^{-1}
// (nc x nc, row-major, upper part zero) followed by W_s = L21 L11^{-1} (m x nc, row-major).
// With t_s = r_s - (updates from descendants):
//   forward   y_s = Linv_s t_s,  updates to the rows R_s: u_s = L21 y_s = W_s t_s
//   backward  x_s = Linv_s^T y_s - W_s^T x_{R_s}
// so one level costs two phases forward (gather t; then y and u together) and one backward.
struct ColRec {
    int32_t off, c0nc, jjm, ridx;
};
__device__ inline ColRec load_col(const int32_t *__restrict__ rec, int i) {
    const int4 v = reinterpret_cast<const int4 *>(rec)[i];
    return ColRec{v.x, v.y, v.z, v.w};
}
__device__ inline int hi16(int32_t w) { return (int)((uint32_t)w >> 16); }
__device__ inline int lo16(int32_t w) { return (int)((uint32_t)w & 0xFFFFu); }

// Forward substitution of one subgraph, R right-hand sides interleaved in LDS.
// In: vec = right side.  Out: vec = y = L^{-1} (right side); tmp, ubuf: scratch.  Level by level,
// leaves first:
//   (a) t_i = vec_i minus the update entries that descendant supernodes left for row i (one thread
//       per column of the level, summed in a fixed order);
//   (b) [y_s; u_s] = V_s t_s for every supernode s of the level, one thread per row of V_s: the
//       level's columns (rows of Linv, results y_i to vec) and then its update entries (rows of W,
//       results u to the update slots), all rows of the level dealt to the threads at once.  A thread
//       runs over the columns j of its supernode; threads on consecutive rows of one supernode read
//       consecutive entries of column j (V_s is stored by columns), so the loads are coalesced.
// Ends with a barrier.
template <typename T, int R>
__device__ void forward_subst(const ClassDev &C, const DevSym &S, const T *__restrict__ Vk, T *vec, T *tmp, T *ubuf) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int32_t *lev_c0 = S.lev_c0 + C.o_lev, *lev_u = S.lev_u + C.o_lev;
    const int32_t *seg_ptr = S.seg_ptr + C.o_colp;
    const uint16_t *seg_u = S.seg_u + C.o_seg;
    const int32_t *colrec = S.colrec + 4 * (int64_t)C.o_col, *urec = S.urec + 4 * (int64_t)C.o_ridx;
    for (int lv = 0; lv < C.nlev; ++lv) {
        const int cb = lev_c0[lv], ce = lev_c0[lv + 1];
        for (int i = cb + tid; i < ce; i += nt) {
            T acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = vec[i * R + c];
            for (int q = seg_ptr[i]; q < seg_ptr[i + 1]; ++q) {
                const T *u = ubuf + seg_u[q] * R;
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] -= u[c];
            }
#pragma unroll
            for (int c = 0; c < R; ++c) tmp[i * R + c] = acc[c];
        }
        __syncthreads();
        const int ub = lev_u[lv], ncol = ce - cb, nrow = ncol + (lev_u[lv + 1] - ub);
        for (int task = tid; task < nrow; task += nt) {
            // one record per row: {block offset, c0<<16|nc, row<<16|m, ridx offset}
            const ColRec r = load_col(task < ncol ? colrec : urec, task < ncol ? cb + task : ub + task - ncol);
            const int nc = lo16(r.c0nc), i = hi16(r.jjm), f = nc + lo16(r.jjm), jn = i < nc ? i + 1 : nc;
            const T *Vs = Vk + r.off;
            const T *t = tmp + hi16(r.c0nc) * R;
            T acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = 0;
            for (int j0 = 0; j0 < jn; j0 += 16) {  // sixteen loads in flight together
                T v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int j = j0 + q < jn ? j0 + q : jn - 1;
                    v[q] = Vs[vcol(f, j) + (i - j)];
                }
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (j0 + q < jn)
#pragma unroll
                        for (int c = 0; c < R; ++c) acc[c] += v[q] * t[(j0 + q) * R + c];
            }
            T *out = task < ncol ? vec + (cb + task) * R : ubuf + (ub + task - ncol) * R;
#pragma unroll
            for (int c = 0; c < R; ++c) out[c] = acc[c];
        }
        __syncthreads();
    }
}

// Backward substitution of one subgraph, root level first: x_s = Linv^T y_s - W^T x_{R_s}, i.e. for
// every column j of s, x_j = (column j of V_s) . [y_s; -x_{R_s}] over its rows j .. f - 1.  One
// thread per column of the level; the column's entries are contiguous (V_s is stored by columns) and
// read sixteen at a time.  In: vec = y.  Out: tmp = x.  Ends with a barrier.
template <typename T, int R>
__device__ void backward_subst(const ClassDev &C, const DevSym &S, const T *__restrict__ Vk, const T *vec, T *tmp) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int32_t *lev_c0 = S.lev_c0 + C.o_lev, *colrec = S.colrec + 4 * (int64_t)C.o_col;
    const uint16_t *ridx = S.ridx + C.o_ridx;
    for (int lv = C.nlev - 1; lv >= 0; --lv) {
        const int cb = lev_c0[lv], ce = lev_c0[lv + 1];
        for (int jg = cb + tid; jg < ce; jg += nt) {
            const ColRec r = load_col(colrec, jg);
            const int c0 = hi16(r.c0nc), nc = lo16(r.c0nc), j = hi16(r.jjm), m = lo16(r.jjm);
            const T *lcol = Vk + r.off + vcol(nc + m, j);  // Linv[j .. nc)[j], then W[0 .. m)[j]
            const T *wcol = lcol + (nc - j);
            const uint16_t *rr = ridx + r.ridx;
            T acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = 0;
            for (int k0 = 0; k0 < nc - j; k0 += 16) {  // Linv^T y: sixteen loads in flight
                T v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) v[q] = k0 + q < nc - j ? lcol[k0 + q] : (T)0;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int row = k0 + q < nc - j ? c0 + j + k0 + q : c0 + j;
#pragma unroll
                    for (int c = 0; c < R; ++c) acc[c] += v[q] * vec[row * R + c];
                }
            }
            for (int q0 = 0; q0 < m; q0 += 16) {  // - W^T x_R
                T v[16];
                int ri[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {  // past m: a zero weight on a row that holds a finished x
                    v[q] = q0 + q < m ? wcol[q0 + q] : (T)0;
                    ri[q] = rr[q0 + q < m ? q0 + q : m - 1];
                }
#pragma unroll
                for (int q = 0; q < 16; ++q)
#pragma unroll
                    for (int c = 0; c < R; ++c) acc[c] -= v[q] * tmp[ri[q] * R + c];
            }
#pragma unroll
            for (int c = 0; c < R; ++c) tmp[jg * R + c] = acc[c];
        }
        __syncthreads();
    }
}

// Forward and backward substitution.  In: vec = right side.  Out: tmp = x, vec = y.
template <typename T, int R>
__device__ void trisolve(const ClassDev &C, const DevSym &S, const T *__restrict__ Vk, T *vec, T *tmp, T *ubuf) {
    forward_subst<T, R>(C, S, Vk, vec, tmp, ubuf);
    backward_subst<T, R>(C, S, Vk, vec, tmp);
}

template <typename T>
__device__ inline T cpl_y(const DevSub &D, int e);
template <>
__device__ inline double cpl_y<double>(const DevSub &D, int e) { return D.cpl_y64[e]; }
template <>
__device__ inline float cpl_y<float>(const DevSub &D, int e) { return D.cpl_y32[e]; }

// One VTM sweep.  flags: kWriteX stores the local solutions; kNoWaves leaves o_next untouched
// (a read-only solve with the current incoming waves); kZeroWaves ignores o_prev (a = 0); kWriteY
// stores the forward result y = L^{-1} (right side) in yout (layout of the local solutions).
// Vectors are laid out in groups of R right-hand sides; a workgroup takes RS of them (the RS-wide
// block rb of group g), so that its LDS -- right side / y, t / x and the update slots, RS values each
// per entry -- fits the CU when the subgraphs are large.
template <typename T, int R, int RS>
__global__ __launch_bounds__(512) void k_sweep(DevSym S, DevSub D, int64_t nsplit, int64_t nports,
                                               const T *__restrict__ vals, const T *__restrict__ bsplit,
                                               const int32_t *__restrict__ twin, const T *__restrict__ invz,
                                               const T *__restrict__ o_prev, T *__restrict__ o_next,
                                               T *__restrict__ xloc, T *__restrict__ yout, int flags) {
    static_assert(RS <= R && R % RS == 0, "right-hand-side block");
    constexpr int NB = R / RS;
    extern __shared__ char smraw[];
    const int k = sub_of_block(D, blockIdx.x), g = blockIdx.y / NB, rb = (blockIdx.y % NB) * RS, tid = threadIdx.x,
              nt = blockDim.x;
    if (sub_inactive(D, k)) return;
    const ClassDev C = S.cls[D.cls[k]];
    const int nk = C.nk;
    T *vec = reinterpret_cast<T *>(smraw);  // right side, then y (forward result)
    T *tmp = vec + (size_t)nk * RS;         // t during the forward pass, x during the backward pass
    T *ubuf = tmp + (size_t)nk * RS;        // update entries W_s t_s of every R_s row
    const T *Vk = vals + D.val[k];
    const int64_t xo = ((int64_t)g * nsplit + D.x[k]) * R + rb;
    const T *bs = bsplit + xo;
    const int64_t wo = (int64_t)g * nports * R + rb;
    const bool zero_waves = flags & kZeroWaves;

    // right side of (5.8): split source + Z^{-1} * incoming wave at every port (with coupled VTLs the
    // off-diagonal entries of Z_j^{-1} add the incoming waves of the coupled ports)
    for (int i = tid; i < nk * RS; i += nt) vec[i] = bs[(i / RS) * R + i % RS];
    __syncthreads();
    const int pg0 = D.pg_ptr[k], pg1 = D.pg_ptr[k + 1];
    if (!zero_waves) {
        for (int q = pg0 + tid; q < pg1; q += nt) {
            const int pos = D.pg_pos[q], pb = D.pg_beg[q], pc = D.pg_cnt[q];
            T acc[RS];
#pragma unroll
            for (int c = 0; c < RS; ++c) acc[c] = vec[pos * RS + c];
            for (int j = 0; j < pc; ++j) {
                const T iz = invz[pb + j];
                const T *a = o_prev + wo + (int64_t)twin[pb + j] * R;
#pragma unroll
                for (int c = 0; c < RS; ++c) acc[c] += a[c] * iz;
                if (D.cpl_ptr)
                    for (int e = D.cpl_ptr[pb + j]; e < D.cpl_ptr[pb + j + 1]; ++e) {
                        const T y = cpl_y<T>(D, e);
                        const T *aq = o_prev + wo + (int64_t)D.cpl_tw[e] * R;
#pragma unroll
                        for (int c = 0; c < RS; ++c) acc[c] += aq[c] * y;
                    }
            }
#pragma unroll
            for (int c = 0; c < RS; ++c) vec[pos * RS + c] = acc[c];
        }
    }
    __syncthreads();
    trisolve<T, RS>(C, S, Vk, vec, tmp, ubuf);
    // outgoing waves o_p = 2 u_p - a_p
    if (!(flags & kNoWaves)) {
        for (int q = pg0 + tid; q < pg1; q += nt) {
            const int pos = D.pg_pos[q], pb = D.pg_beg[q], pc = D.pg_cnt[q];
            for (int j = 0; j < pc; ++j) {
                const T *a = o_prev + wo + (int64_t)twin[pb + j] * R;
                T *o = o_next + wo + (int64_t)(pb + j) * R;
#pragma unroll
                for (int c = 0; c < RS; ++c) o[c] = (T)2 * tmp[pos * RS + c] - (zero_waves ? (T)0 : a[c]);
            }
        }
    }
    if (flags & kWriteX) {
        T *xo_ = xloc + xo;
        for (int i = tid; i < nk * RS; i += nt) xo_[(i / RS) * R + i % RS] = tmp[i];
    }
    if (flags & kWriteY) {
        T *yo_ = yout + xo;
        for (int i = tid; i < nk * RS; i += nt) yo_[(i / RS) * R + i % RS] = vec[i];
    }
}

// Local solve of a convergence test from the port Green's columns Y = L^{-1} E (E: unit columns of
// the port vertices, in the plan's port order) kept by the factorisation:
//   x = K^{-1} (b~ + E w) = L^{-T} (y_b + Y w),  w = Z^{-1} a summed per port vertex,
// with y_b = L^{-1} b~ stored by the zero-wave solve of the current source.  One parallel phase and
// the backward substitution replace the level-by-level forward substitution.  Y rows of supernode
// s (nc_s x w_s, row-major) live in its region of the Green workspace: after its port front in FP64,
// column-major at y32_pos in the FP32 copy.
template <typename T, int R>
__global__ __launch_bounds__(512) void k_ysolve(DevSym S, DevSub D, DevGreen Gp, const T *__restrict__ Yw,
                                                int64_t nsplit, int64_t nports, const T *__restrict__ vals,
                                                const T *__restrict__ yb, const int32_t *__restrict__ twin,
                                                const T *__restrict__ invz, const T *__restrict__ o_in,
                                                T *__restrict__ xloc) {
    extern __shared__ char smraw[];
    const int k = sub_of_block(D, blockIdx.x), g = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
    if (sub_inactive(D, k)) return;
    const ClassDev C = S.cls[D.cls[k]];
    const int nk = C.nk;
    T *vec = reinterpret_cast<T *>(smraw);  // y
    T *tmp = vec + (size_t)nk * R;          // x
    T *wsrt = tmp + (size_t)nk * R;         // w per port vertex, plan order
    const T *Vk = vals + D.val[k];
    const int64_t xo = ((int64_t)g * nsplit + D.x[k]) * R, wo = (int64_t)g * nports * R;
    for (int i = tid; i < nk * R; i += nt) vec[i] = yb[xo + i];
    const int pg0 = D.pg_ptr[k], p = D.pg_ptr[k + 1] - pg0;
    for (int a = tid; a < p; a += nt) {
        const int q = pg0 + Gp.perm[pg0 + a];
        const int pb = D.pg_beg[q], pc = D.pg_cnt[q];
        T acc[R];
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] = 0;
        for (int j = 0; j < pc; ++j) {
            const T iz = invz[pb + j];
            const T *av = o_in + wo + (int64_t)twin[pb + j] * R;
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] += av[c] * iz;
        }
#pragma unroll
        for (int c = 0; c < R; ++c) wsrt[a * R + c] = acc[c];
    }
    __syncthreads();
    const int4 *pl = Gp.sn + Gp.base[k];
    const int32_t *col_sn = S.col_sn + C.o_col, *sn_c0 = S.sn_c0 + C.o_sn, *sn_nc = S.sn_nc + C.o_sn,
                  *sn_m = S.sn_m + C.o_sn;
    const T *Yk = Yw + Gp.wso[k];
    for (int col = tid; col < nk; col += nt) {  // y += Y w, one factor column (row of Y) per thread
        const int s = col_sn[col];
        const int4 e = pl[s];
        const int w = (int)((uint32_t)e.y >> 16), pc0 = e.y & 0xFFFF;
        if (w == 0) continue;
        const int f = sn_nc[s] + sn_m[s], row = col - sn_c0[s];
        const T *wr = wsrt + (size_t)pc0 * R;
        T acc[R];
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] = 0;
        if (sizeof(T) == 4) {
            // FP32 columns (y32_pos): the lanes of a supernode read consecutive rows of each column
            // (coalesced), eight columns in flight; the weights are LDS broadcasts
            const T *yc = Yk + y32_pos(e.x, sn_nc[s], row, 0);
            const int ldc = sn_nc[s];
            for (int a0 = 0; a0 < w; a0 += 8) {
                T yv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) yv[q] = a0 + q < w ? yc[(int64_t)(a0 + q) * ldc] : (T)0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const T *wa = wr + (size_t)(a0 + q < w ? a0 + q : w - 1) * R;
#pragma unroll
                    for (int c = 0; c < R; ++c) acc[c] += yv[q] * wa[c];
                }
            }
        } else {
            const T *yr = Yk + e.x + (int64_t)f * w + (int64_t)row * w;
            for (int a0 = 0; a0 < w; a0 += 16) {  // sixteen loads in flight before the first product
                T yv[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) yv[q] = a0 + q < w ? yr[a0 + q] : (T)0;
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (a0 + q < w)
#pragma unroll
                        for (int c = 0; c < R; ++c) acc[c] += yv[q] * wr[(a0 + q) * R + c];
            }
        }
#pragma unroll
        for (int c = 0; c < R; ++c) vec[col * R + c] += acc[c];
    }
    __syncthreads();
    backward_subst<T, R>(C, S, Vk, vec, tmp);
    T *xo_ = xloc + xo;
    for (int i = tid; i < nk * R; i += nt) xo_[i] = tmp[i];
}

// Port Green's functions G_k = R_k K_k^{-1} R_k^T (R_k selects the port vertices), FP64:
// column j of G_k is the port part of K_k^{-1} e_{v(j)}; blockIdx.y picks RHS columns j.
template <int R>
__global__ __launch_bounds__(256) void k_green(DevSym S, DevSub D, const double *__restrict__ vals,
                                               const int64_t *__restrict__ goff, double *__restrict__ G) {
    extern __shared__ char smraw[];
    const int k = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const ClassDev C = S.cls[D.cls[k]];
    const int nk = C.nk;
    const int pg0 = D.pg_ptr[k], p = D.pg_ptr[k + 1] - pg0;
    const int j0 = blockIdx.y * R;
    if (j0 >= p) return;  // uniform across the workgroup
    double *vec = reinterpret_cast<double *>(smraw);
    double *tmp = vec + (size_t)nk * R;
    double *ubuf = tmp + (size_t)nk * R;
    for (int i = tid; i < nk * R; i += nt) vec[i] = 0.0;
    __syncthreads();
    if (tid < R && j0 + tid < p) vec[D.pg_pos[pg0 + j0 + tid] * R + tid] = 1.0;
    __syncthreads();
    trisolve<double, R>(C, S, vals + D.val[k], vec, tmp, ubuf);
    double *Gk = G + goff[k];
    const int nb = (p + 15) >> 4;
    for (int idx = tid; idx < R * p; idx += nt) {
        const int c = idx / p, q = idx - c * p;
        if (j0 + c < p) {
            const int64_t e = gpack_index(nb, j0 + c, q);
            if (e >= 0) Gk[e] = tmp[D.pg_pos[pg0 + q] * R + c];
        }
    }
}

// Diagonal of every G_k (one entry per port vertex), from the packed layout.
__global__ void k_gdiag(DevSub D, const int64_t *__restrict__ goff, const double *__restrict__ G,
                        double *__restrict__ gd) {
    const int k = blockIdx.x;
    const int pg0 = D.pg_ptr[k], p = D.pg_ptr[k + 1] - pg0, nb = (p + 15) >> 4;
    for (int j = threadIdx.x; j < p; j += blockDim.x) gd[pg0 + j] = G[goff[k] + gpack_index(nb, j, j)];
}

// Input impedance of every port (Definition 7.1) with the other ports of its subgraph terminated by
// their Z: with g the diagonal entry of G_k at the port's vertex, r = 1 / (1/g - 1/Z_p); +inf where the
// port's own termination is what makes K_k definite (1/g - 1/Z_p <= 1e-14 / g).  One workgroup per
// subgraph, one thread per port.
__global__ void k_rin(DevSub D, const int64_t *__restrict__ goff, const double *__restrict__ G,
                      const double *__restrict__ invz, double *__restrict__ r) {
    const int k = blockIdx.x;
    const int p = D.pg_ptr[k + 1] - D.pg_ptr[k], nb = (p + 15) >> 4;
    const double *Gk = G + goff[k];
    for (int t = D.port_ptr[k] + threadIdx.x; t < D.port_ptr[k + 1]; t += blockDim.x) {
        const int i = D.port_pg[t];
        const double g = Gk[gpack_index(nb, i, i)];
        const double d = 1.0 / g - invz[t];
        r[t] = d > 1e-14 / g ? 1.0 / d : __builtin_inf();
    }
}

// c[g][q][c] = K^{-1} b~ at the port vertices (local solutions of a zero-wave solve).
template <typename T>
__global__ void k_gather_ports(DevSub D, int64_t nsplit, int32_t npg, int32_t R, const T *__restrict__ xloc,
                               T *__restrict__ cport) {
    const int k = sub_of_block(D, blockIdx.x), g = blockIdx.y;
    if (sub_inactive(D, k)) return;
    const int pg0 = D.pg_ptr[k], pg1 = D.pg_ptr[k + 1];
    const int64_t xo = ((int64_t)g * nsplit + D.x[k]) * R;
    for (int idx = threadIdx.x; idx < (pg1 - pg0) * R; idx += blockDim.x) {
        const int q = idx / R, c = idx - q * R;
        cport[((int64_t)g * npg + pg0 + q) * R + c] = xloc[xo + D.pg_pos[pg0 + q] * R + c];
    }
}

// Port-reduced sweep: u = c + G (Z^{-1} a) on the port vertices, then o_p = 2 u - a_p.
// G_k is symmetric; it is stored as its lower block triangle of 16 x 16 blocks (diagonal blocks in
// full, rows and columns padded with zeros to nb = ceil(p / 16) blocks), block column by block
// column (see gpack_index and gblk_pos), so that the blocks of G_k are read in storage order.
//
// One wave per (subgraph, RHS group): workgroup b takes subgraph gorder[b] (largest G_k first, so that
// the longest waves start early and the short ones fill the tail).  The wave streams its blocks with
// PF of them in flight.  Lane l = 16 q + m holds B[m][4 q .. 4 q + 4) of a block B = G[I][J] (one
// or two 16-byte loads).  For every block, y_I += B x_J runs on the matrix cores: four
// v_mfma_*_16x16x4 whose A operand is the lane's four entries and whose B operand is x_J (column
// c < R of the 16 x 16 operand holds right-hand side c, the rest zero); the product is added to y_I
// in LDS.  For an off-diagonal block, y_J += B^T x_I runs on the vector units: lane (m, q) adds
// B[m][4 q + kk] x_I[m][c] into registers for the whole block column, and the 16 lanes of each q
// are summed once per column (DPP row rotations).  A single wave adds into y in program order, so
// the result does not depend on timing.  LDS holds Z^{-1} a and y, 2 pp R values.
template <typename T> struct Quad;
template <> struct Quad<float> {
    float4 v;
    __device__ void load(const float *p) { v = *reinterpret_cast<const float4 *>(p); }
    __device__ float operator[](int i) const { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
};
template <> struct Quad<double> {
    double2 a, b;
    __device__ void load(const double *p) {
        a = reinterpret_cast<const double2 *>(p)[0];
        b = reinterpret_cast<const double2 *>(p)[1];
    }
    __device__ double operator[](int i) const { return i == 0 ? a.x : i == 1 ? a.y : i == 2 ? b.x : b.y; }
};

// Sum of v[0 .. N) over the 16 lanes of each DPP row, scattered: level by level (lane bits 3, 0, 1,
// 2) a lane keeps the lower or upper half of its values, by its bit, and adds the partner's copy of
// that half.  With N >= 16, lane m ends with the complete sums of the N / 16 values
// j0 + [0, N / 16) in v[0 ..), j0 = scatter_base<N>(m).  With N < 16 the last levels add the single
// value of both partners, so that every lane of a group holds the sum; the group's lane with the
// unused bits zero writes it (scatter_writer<N>).
template <typename T, int N, int L = 0>
__device__ inline void row16_reduce_scatter(T (&v)[N], int m) {
    if constexpr (L < 4) {
        constexpr int X = L == 0 ? 8 : L == 1 ? 1 : L == 2 ? 2 : 4;
        constexpr int S = L == 0 ? 3 : L == 1 ? 0 : L == 2 ? 1 : 2;
        constexpr int C = (N >> L) > 1 ? (N >> L) : 1;  // values held before this level
        if constexpr (C > 1) {
            const bool up = (m >> S) & 1;
#pragma unroll
            for (int i = 0; i < C / 2; ++i) {
                const T keep = up ? v[C / 2 + i] : v[i], send = up ? v[i] : v[C / 2 + i];
                v[i] = keep + lane_xor<X>(send);
            }
        } else {
            v[0] += lane_xor<X>(v[0]);
        }
        row16_reduce_scatter<T, N, L + 1>(v, m);
    }
}
template <int N>
__device__ inline int scatter_base(int m) {
    int j0 = 0, c = N;
    const int bits[4] = {3, 0, 1, 2};
#pragma unroll
    for (int L = 0; L < 4; ++L)
        if (c > 1) {
            if ((m >> bits[L]) & 1) j0 += c / 2;
            c /= 2;
        }
    return j0;
}
template <int N>
__device__ inline bool scatter_writer(int m) {
    int c = N;
    const int bits[4] = {3, 0, 1, 2};
    bool w = true;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        if (c <= 1 && ((m >> bits[L]) & 1)) w = false;
        c = c > 1 ? c / 2 : 1;
    }
    return w;
}

// 16 x 16 x 4 matrix-core step D += A B: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator register i of lane l holds D[row(l / 16, i)][l % 16], with row 4 (l / 16) + i for the
// FP32 instruction and 4 i + l / 16 for the FP64 one.
template <typename T> struct Mma;
template <> struct Mma<float> {
    typedef f32x4 acc;
    __device__ static acc step(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int q, int i) { return 4 * q + i; }
    __device__ static int yrow(int r) { return r; }  // accumulator rows 4 q + i are consecutive
};
template <> struct Mma<double> {
    typedef f64x4 acc;
    __device__ static acc step(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int q, int i) { return 4 * i + q; }
    __device__ static int yrow(int r) { return 4 * (r & 3) + (r >> 2); }  // stores row 4 i + q at 4 q + i
};

// Four consecutive values from or to LDS in one 16-byte access (two for doubles); p is 16-byte aligned.
__device__ inline void lds_get4(const float *p, float (&v)[4]) {
    const float4 t = *reinterpret_cast<const float4 *>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ inline void lds_put4(float *p, const float (&v)[4]) { *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]); }
__device__ inline void lds_get4(const double *p, double (&v)[4]) {
    const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ inline void lds_put4(double *p, const double (&v)[4]) {
    reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}

template <typename T, int R, int W>
__global__ __launch_bounds__(W == 1 ? 256 : 64 * W) void k_schur(DevSub D, int32_t nslots, int32_t team_bytes, int32_t npg,
                                                              int64_t nports, const T *__restrict__ G,
                                                              const int64_t *__restrict__ goff, const T *__restrict__ cport,
                                                              const int32_t *__restrict__ twin, const T *__restrict__ invz,
                                                              const T *__restrict__ o_prev, T *__restrict__ o_next) {
    static_assert(R == 1 || R == 2 || R == 4 || R == 8, "right-hand sides per wave");
    extern __shared__ char smem_all[];
    constexpr int PF = 4;                         // blocks in flight (4 KB FP32, 8 KB FP64)
    constexpr int U = 4;                          // ports per lane whose loads are issued together
    constexpr int NV = 4 * R;                     // column partial sums per lane, index c * 4 + kk
    typedef typename Mma<T>::acc Acc;
    // A team of W waves sweeps one subgraph.  With one wave per team, a workgroup holds several
    // independent teams (blockDim.x / 64 of them, each with its own LDS), so that a CU is not limited
    // by the number of workgroups it can hold; their syncs are wave-level.
    const int nt = 64 * W, team = W == 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) : 0;
    const int slot = blockIdx.x * ((int)blockDim.x / nt) + team;
    if (slot >= nslots) return;
    const int k = D.sub_list ? D.sub_list[slot] : D.gorder[slot], g = blockIdx.y, tid = (int)threadIdx.x - team * nt;
    if (sub_inactive(D, k)) return;
    char *smraw = smem_all + (size_t)team * team_bytes;
    auto team_sync = [] {
        if constexpr (W == 1) wave_sync();
        else __syncthreads();
    };
    const int lane = tid & 63, m = lane & 15, q = lane >> 4;
    const int wv = W == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pg0 = D.pg_ptr[k], p = D.pg_ptr[k + 1] - pg0;
    const int nb = (p + 15) >> 4, pp = nb * 16;
    const int ps = pp + 4;                         // row stride of y (staggers the LDS banks of the RHS)
    const int64_t wo = (int64_t)g * nports * R;
    T *xz = reinterpret_cast<T *>(smraw);  // Z^{-1} a per port vertex [pp][R], entries at xzi
    T *y = xz + (size_t)pp * R;            // per wave: G Z^{-1} a from its blocks [W][R][ps], rows in yrow order
    T *scr = y;                            // before y: Z^{-1} a per port [np_k][R]
    T *ydummy = y + (size_t)W * ps * R;    // after y (over the scratch): 4 values per lane for the unused lanes
    // With 8 RHS, the two halves of a row of xz swap places in every other group of 4 rows, so that
    // the 16-byte reads of 8 consecutive rows fall in distinct LDS banks.
    auto xzi = [](int r, int c) { return r * R + (R == 8 ? (c ^ (((r >> 2) & 1) << 2)) : c); };
    const T *Gl = G + goff[k] + 4 * lane;  // B[m][4 q .. 4 q + 4), see gblk_pos
    // With W = 2 the two waves take alternate pairs of block columns (0 3 4 7 8 ... and 1 2 5 6 ...,
    // about equal numbers of blocks), each adding into its own copy of y; the copies are summed in a
    // fixed order at the end.
    auto owner = [&](int j) { return W == 1 ? 0 : ((j ^ (j >> 1)) & 1); };
    auto next_col = [&](int j) {  // the owner pattern has period 4: the next own column is 1 to 3 ahead
        if (W == 1) return j + 1;
        return owner(j + 1) == wv ? j + 1 : owner(j + 2) == wv ? j + 2 : j + 3;
    };
    const int col0 = W == 1 ? 0 : (nb > wv ? wv : nb);
    int nblk = 0;
    for (int j = col0; j < nb; j = next_col(j)) nblk += nb - j;
    // load cursor: block (Il, Jl) of this wave's sequence, PF blocks ahead of the one in use, and the
    // offset of block (Jl, Jl) (blocks of a column are consecutive)
    int Jl = col0, Il = col0;
    int64_t coff = ((int64_t)col0 * nb - (int64_t)col0 * (col0 - 1) / 2) * 256;
    // past the wave's last block a slot loads the block after G_k (inside the next G_k or the
    // allocation's one-block padding): an address of its own, so that the load is not merged with a
    // real one, which would make its use wait for that load
    const int64_t past = (int64_t)nb * (nb + 1) / 2 * 256;
    auto next_load = [&]() {
        const int64_t off = Jl < nb ? coff + (int64_t)(Il - Jl) * 256 : past;
        if (Il + 1 < nb) {
            ++Il;
        } else {
            const int Jn = next_col(Jl);
            coff = ((int64_t)Jn * nb - (int64_t)Jn * (Jn - 1) / 2) * 256;
            Jl = Jn;
            Il = Jn;
        }
        return off;
    };
    // Z^{-1} a_p for every port (a_p = o_twin(p)) into the scratch, with the loads of U ports per thread
    // issued before the first of them is used; then xz[v] = the sum over the ports at vertex v, in
    // port order (no LDS atomics: a float atomic costs far more than a read and a write).  The first
    // U ports of each thread keep their twin, vertex and incoming wave in registers for the write-back,
    // and the first vertex records are requested with them.  Loads complete in issue order, so the
    // first ports' loads go out before the G stream starts, which would otherwise sit in front of them.
    const int port0 = D.port_ptr[k], np_k = D.port_ptr[k + 1] - port0;
    int tw0[U], v0r[U], vb0[U], vc0[U];
    T a0[U][R], iz0[U];
    // vertex record (first port, port count) with an unconditional load (a clamped index), so that
    // nothing waits for it before it is used; vertices past p get no ports there
    auto vertex_rec = [&](int v, int &b, int &c) {
        const int vc = v < p ? v : p - 1;
        b = D.pg_beg[pg0 + vc];
        c = D.pg_cnt[pg0 + vc];
    };
    auto port_loads = [&](int t0, int (&tw)[U], int (&vv)[U], T (&iz)[U], T (&a)[U][R]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + nt * u + tid, pt = port0 + (t < np_k ? t : 0);
            tw[u] = twin[pt];
            iz[u] = invz[pt];
            vv[u] = D.port_pg[pt];
        }
        if (t0 == 0)
#pragma unroll
            for (int u = 0; u < U; ++u) vertex_rec(nt * u + tid, vb0[u], vc0[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < R; ++c) a[u][c] = o_prev[wo + (int64_t)tw[u] * R + c];
    };
    auto port_store = [&](int t0, const T (&iz)[U], const T (&a)[U][R]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + nt * u + tid;
            if (t < np_k)
#pragma unroll
                for (int c = 0; c < R; ++c) scr[t * R + c] = a[u][c] * iz[u];
        }
    };
    if (np_k > 0) port_loads(0, tw0, v0r, iz0, a0);
    // Every slot issues one load per refill, past the last block too (see past): with the same number
    // of loads in flight on every path, each use waits only for its own block.  The loads are kept in slot order (scheduling barriers), as the refills are
    // issued: then the queue is in the same order on entry to the loop and around it.
    __builtin_amdgcn_sched_barrier(0);
    Quad<T> pre[PF];
#pragma unroll
    for (int f = 0; f < PF; ++f) {
        pre[f].load(Gl + next_load());
        __builtin_amdgcn_sched_barrier(0);
    }
    if (np_k > 0) port_store(0, iz0, a0);
    for (int t0 = nt * U; t0 < np_k; t0 += nt * U) {
        int tw[U], vv[U];
        T iz[U], a[U][R];
        port_loads(t0, tw, vv, iz, a);
        port_store(t0, iz, a);
    }
    team_sync();
    for (int v0 = 0; v0 < pp; v0 += nt * U) {
        int b0[U], cnt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (v0 == 0) {
                b0[u] = vb0[u];
                cnt[u] = vc0[u];
            } else {
                vertex_rec(v0 + nt * u + tid, b0[u], cnt[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + nt * u + tid, n = v < p ? cnt[u] : 0, t1 = b0[u] - port0;
            T s_[R];
#pragma unroll
            for (int c = 0; c < R; ++c) s_[c] = 0;
            for (int j = 0; j < n; ++j)
#pragma unroll
                for (int c = 0; c < R; ++c) s_[c] += scr[(t1 + j) * R + c];
            if (v < pp)
#pragma unroll
                for (int c = 0; c < R; ++c) xz[xzi(v, c)] = s_[c];
        }
    }
    team_sync();
    for (int i = tid; i < W * ps * R; i += nt) y[i] = 0;
    team_sync();
    // B operand of y_I += B x_J: lane (m, q) gives x_J[4 q + kk][m] for m < R
    T xb[4], xbn[4];
    auto load_xb = [&](T (&d)[4], int J) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) d[kk] = m < R ? xz[xzi(J * 16 + 4 * q + kk, m < R ? m : 0)] : (T)0;
    };
    T tc[NV];  // partial column sums of B^T x_I for the current block column
#pragma unroll
    for (int j = 0; j < NV; ++j) tc[j] = 0;
    // x_I[m][.] of the next block is read one block ahead, into the other of two register sets
    T xi[2][R];
    auto load_xi = [&](T (&xd)[R], int I) {
        const int r = I * 16 + m;
        if constexpr (R == 8) {
            T h0[4], h1[4];
            lds_get4(xz + xzi(r, 0), h0);
            lds_get4(xz + xzi(r, 4), h1);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                xd[c] = h0[c];
                xd[4 + c] = h1[c];
            }
        } else if constexpr (R == 4) {
            T h0[4];
            lds_get4(xz + r * 4, h0);
#pragma unroll
            for (int c = 0; c < 4; ++c) xd[c] = h0[c];
        } else {
#pragma unroll
            for (int c = 0; c < R; ++c) xd[c] = xz[r * R + c];
        }
    };
    // lane (m < R, q) owns y[m][rows of block I at yrow(4 q) .. + 4), the rows of its accumulator;
    // the other lanes (whose products are zero) read and write 4 values of their own.  The product of
    // block b is added to y while block b + 1 is on the matrix cores (the rows of two consecutive
    // blocks of a column differ; with none pending, the write goes to the lane's own 4 values); at the
    // end of a column it is added at once.  No branch separates the matrix-core steps from the
    // vector-unit products of a block, so that they can be interleaved.
    T *yw = y + (size_t)wv * R * ps;
    T *const ydl = ydummy + 4 * tid;
    T *yl = m < R ? yw + m * ps + 4 * q : ydl;
    const int ystep = m < R ? 16 : 0;
    const int j0 = scatter_base<NV>(m);
    const bool writer = scatter_writer<NV>(m);
    // block b's product and y rows live in the register set b % 2 (PF is even, so the slot's parity)
    Acc acc[2] = {Acc{0, 0, 0, 0}, Acc{0, 0, 0, 0}};
    T yv[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    int IP = nb;
    int J = col0, I = col0;
    load_xb(xb, col0 < nb ? col0 : 0);
#pragma unroll
    for (int c = 0; c < R; ++c) xi[0][c] = 0;  // block (0, 0) is diagonal
    for (int b0 = 0; b0 < nblk; b0 += PF) {
#pragma unroll
        for (int f = 0; f < PF; ++f) {
            if (b0 + f < nblk) {
                const int e = f & 1, o = e ^ 1;  // this block's register set, the previous block's
                const Quad<T> vb = pre[f];
                lds_get4(yl + I * ystep, yv[e]);
                acc[e] = Acc{0, 0, 0, 0};
                const T(&xc)[R] = xi[e];  // zero for a diagonal block (its B^T x_I is inside B x_J)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    acc[e] = Mma<T>::step(vb[kk], xb[kk], acc[e]);
#pragma unroll
                    for (int c = 0; c < R; ++c) tc[c * 4 + kk] += vb[kk] * xc[c];
                }
                {  // the previous block's product (one wave owns y: plain read-modify-write)
                    T w[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) w[i] = yv[o][i] + acc[o][i];
                    lds_put4(IP < nb ? yl + IP * ystep : ydl, w);
                }
                const bool last = I + 1 == nb;
                const int In = last ? next_col(J) : I + 1;  // next block's row (its column is J or In)
                load_xi(xi[o], In < nb ? In : nb - 1);
                if (last) {  // end of block column J: this block's product, y_J += the column sums
                    if (In < nb) load_xb(xbn, In);
                    {
                        T w[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) w[i] = yv[e][i] + acc[e][i];
                        lds_put4(yl + I * ystep, w);
                    }
                    IP = nb;
#pragma unroll
                    for (int c = 0; c < R; ++c) xi[o][c] = 0;  // the next block is diagonal
                    row16_reduce_scatter<T, NV>(tc, m);
                    if (writer)
#pragma unroll
                        for (int i = 0; i < (NV >= 16 ? NV / 16 : 1); ++i) {
                            const int jj = j0 + i, c = jj >> 2, kk = jj & 3;
                            T *yj = yw + c * ps + J * 16 + Mma<T>::yrow(4 * q + kk);
                            *yj += tc[i];
                        }
#pragma unroll
                    for (int j = 0; j < NV; ++j) tc[j] = 0;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) xb[kk] = xbn[kk];
                    J = In;
                } else {
                    IP = I;
                }
                I = In;
            }
            pre[f].load(Gl + next_load());
        }
    }
    team_sync();
    // u = c + y at each port vertex; o_p = 2 u - a_p (loads of U ports per lane issued together; the
    // first U ports per lane from the registers kept by the gather)
    for (int t0 = 0; t0 < np_k; t0 += nt * U) {
        int tw[U], v[U];
        T a[U][R], cu[U][R];
        if (t0 == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                tw[u] = tw0[u];
                v[u] = v0r[u];
#pragma unroll
                for (int c = 0; c < R; ++c) a[u][c] = a0[u][c];
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + nt * u + tid, pt = port0 + (t < np_k ? t : 0);
                tw[u] = twin[pt];
                v[u] = D.port_pg[pt];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < R; ++c) a[u][c] = o_prev[wo + (int64_t)tw[u] * R + c];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < R; ++c) cu[u][c] = cport[((int64_t)g * npg + pg0 + v[u]) * R + c];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + nt * u + tid, yr = (v[u] & ~15) + Mma<T>::yrow(v[u] & 15);
            if (t < np_k)
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    T yy = y[c * ps + yr];
#pragma unroll
                    for (int w = 1; w < W; ++w) yy += y[((size_t)w * R + c) * ps + yr];
                    o_next[wo + (int64_t)(port0 + t) * R + c] = (T)2 * (cu[u][c] + yy) - a[u][c];
                }
        }
    }
}

// ------------------------------------------------------------ persistent port-reduced sweeps
//
// One launch runs nsw sweeps of the port-reduced map (k_schur's arithmetic, FP32).  Workgroup (k, g)
// keeps its blocks of G_k in registers for the whole launch, so a sweep moves only the waves.
// Sweeps are ordered by the waves themselves: every outgoing wave is published as one 64-bit word
// {sweep tag, FP32 value} by a relaxed agent-scope atomic store into the buffer of its sweep's
// parity, and a workgroup starts sweep s once each of its incoming words carries tag s - 1 (a
// single-copy-atomic word needs no separate flag or fence).  Two buffers suffice: the word of sweep
// s overwrites the one of sweep s - 2, which the twin's owner read during its sweep s - 1, before
// it published the sweep s - 1 word this workgroup waited for.  Neighbours thus stay within one
// sweep of each other.  A launch starting at tag t0 first publishes its starting waves with tag t0
// and then awaits tags t0 .. t0 + nsw - 1 only; no word left from earlier launches carries one of
// them (the host advances t0 by nsw + 2 per launch, restarts it at 1 only past 2^29, and zeroes a new
// buffer; tag 0 is never awaited).
// All workgroups must be resident at once (cooperative launch).  Every wait
// is bounded: a wait that exceeds spin_limit polls raises *abort, every other wait then gives up
// too, and the launch runs to its end with the host reporting the error.

__device__ inline unsigned long long load_word(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_word(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long tag_word(int tag, float v) {
    return ((unsigned long long)(unsigned)tag << 32) | (unsigned long long)__float_as_uint(v);
}

// Wait until the word at w carries tag want (re-reading it), bounded by spin_limit polls or an abort.
__device__ inline unsigned long long await_word(const unsigned long long *w, unsigned long long v, int want,
                                                int spin_limit, int32_t *abort_flag) {
    int spins = 0;
    while ((int)(v >> 32) != want) {
        ++spins;
        if (spins > spin_limit ||
            ((spins & 63) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = load_word(w);
    }
    return v;
}

// Workgroup (k, g), 256 threads: thread t owns a 4 x 16 tile of G_k (rows 4 (t / 8) .. + 4,
// columns 16 (t % 8) .. + 16; zero beyond p_k), expanded once per launch from the packed blocks into
// 64 registers; p_k <= 128.  Per sweep: (A) one thread per port awaits its incoming word; (A2) one
// thread per port vertex forms Z^{-1} a; (B) each thread multiplies its tile by its 16 entries of
// Z^{-1} a (four 16-byte LDS reads), the 8 threads of a row group add their partial sums (DPP quad
// permutations, then a swizzle), and thread 4 (t / 8) + j writes the outgoing waves of row 4 (t / 8)
// + j's port vertex.
template <int R>
__global__ __launch_bounds__(256, 4) void k_schur_persist(DevSub D, int32_t npg, int64_t nports, int32_t max_np,
                                                          const float *__restrict__ G,
                                                          const int64_t *__restrict__ goff,
                                                          const float *__restrict__ cport,
                                                          const int32_t *__restrict__ twin,
                                                          const float *__restrict__ invz, unsigned long long *tw,
                                                          float *plain0, float *plain1, int32_t t0, int32_t nsw,
                                                          int32_t cur0, int32_t spin_limit, int32_t *abort_flag) {
    extern __shared__ __attribute__((aligned(16))) char smraw[];
    const int k = blockIdx.x, g = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
    // a converged system's workgroups leave at once: their twins are in the same system
    if (sub_inactive(D, k)) return;
    const int pg0 = D.pg_ptr[k], p = D.pg_ptr[k + 1] - pg0;
    const int nb = (p + 15) >> 4;
    const int64_t wo = (int64_t)g * nports * R, bstride = (int64_t)gridDim.y * nports * R;
    // LDS, double-buffered by sweep parity: xz [2][128][R], a [2][max_np][R]; Z^{-1} and twin per port
    float *xz2 = reinterpret_cast<float *>(smraw);
    float *al2 = xz2 + (size_t)2 * 128 * R;
    float *izl = al2 + (size_t)2 * max_np * R;
    int *twl = reinterpret_cast<int *>(izl + max_np);
    __shared__ int stop[2];
    const int port0 = D.port_ptr[k], np_k = D.port_ptr[k + 1] - port0;
    const float *Gk = G + goff[k];
    const int rg = tid >> 3, cg = tid & 7;   // rows 4 rg .. + 4, columns 16 cg .. + 16
    float gr[4][16];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int i = 4 * rg + rr, j = 16 * cg + cc;
            float v = 0.f;
            if (i < p && j < p) {
                const int I = i >> 4, J = j >> 4;
                v = I >= J ? Gk[((int64_t)J * nb - (int64_t)J * (J - 1) / 2 + (I - J)) * 256 + gblk_pos(i & 15, j & 15)]
                           : Gk[((int64_t)I * nb - (int64_t)I * (I - 1) / 2 + (J - I)) * 256 + gblk_pos(j & 15, i & 15)];
            }
            gr[rr][cc] = v;
        }
    // this thread's port vertex for Z^{-1} a (q = tid), and for the output (row 4 rg + cg, cg < 4)
    const int orow = 4 * rg + cg;
    const bool outer = cg < 4 && orow < p;
    int qb = 0, qc = 0, rb = 0, rc = 0;
    float cq[R];
    if (tid < p) {
        qb = D.pg_beg[pg0 + tid] - port0;
        qc = D.pg_cnt[pg0 + tid];
    }
    if (outer) {
        rb = D.pg_beg[pg0 + orow] - port0;
        rc = D.pg_cnt[pg0 + orow];
#pragma unroll
        for (int c = 0; c < R; ++c) cq[c] = cport[((int64_t)g * npg + pg0 + orow) * R + c];
    }
    for (int t = tid; t < np_k; t += nt) {
        twl[t] = twin[port0 + t];
        izl[t] = invz[port0 + t];
    }
    for (int e = tid; e < 2 * 128 * R; e += nt) xz2[e] = 0.f;  // rows >= p stay zero
    // the starting waves of this workgroup's ports, published with tag t0 by the threads that publish
    // them at every sweep (so each word's stores keep program order)
    if (outer) {
        const float *start = cur0 == 0 ? plain0 : plain1;
        unsigned long long *dst = tw + (int64_t)(t0 & 1) * bstride + wo;
        for (int j = 0; j < rc; ++j) {
            const int64_t o = (int64_t)(port0 + rb + j) * R;
#pragma unroll
            for (int c = 0; c < R; ++c) store_word(dst + o + c, tag_word(t0, start[wo + o + c]));
        }
    }
    __syncthreads();
    for (int i = 1; i <= nsw; ++i) {
        const int s = t0 + i, par = i & 1;
        float *xz = xz2 + (size_t)par * 128 * R, *al = al2 + (size_t)par * max_np * R;
        // A: incoming words of sweep s - 1, one thread per port (all loads issued before any wait)
        const unsigned long long *src = tw + (int64_t)((s - 1) & 1) * bstride + wo;
        if (tid == 0) stop[par] = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int t = tid; t < np_k; t += nt) {
            const unsigned long long *w = src + (int64_t)twl[t] * R;
            unsigned long long v[R];
#pragma unroll
            for (int c = 0; c < R; ++c) v[c] = load_word(w + c);
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const unsigned long long x = await_word(w + c, v[c], s - 1, spin_limit, abort_flag);
                al[t * R + c] = __uint_as_float((unsigned)(x & 0xFFFFFFFFull));
            }
        }
        __syncthreads();
        if (stop[par]) return;  // uniform: the whole workgroup leaves
        // A2: xz = sum over the port vertex's ports of Z^{-1} a (fixed order)
        if (tid < p) {
            float acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = 0.f;
            for (int j = 0; j < qc; ++j)
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] += al[(qb + j) * R + c] * izl[qb + j];
#pragma unroll
            for (int c = 0; c < R; ++c) xz[tid * R + c] = acc[c];
        }
        __syncthreads();
        // B: tile times its 16 entries of xz, row-group sums over the 8 threads, outgoing waves
        float acc[4][R];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int c = 0; c < R; ++c) acc[rr][c] = 0.f;
        const float4 *x4 = reinterpret_cast<const float4 *>(xz + (size_t)16 * cg * R);  // 16-byte LDS reads
#pragma unroll
        for (int q4 = 0; q4 < 4 * R; ++q4) {
            const float4 xv = x4[q4];
            const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int cc = (4 * q4 + e) / R, c = (4 * q4 + e) % R;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) acc[rr][c] += gr[rr][cc] * xs[e];
            }
        }
        // reduce-scatter over the 8 threads of the row group: thread cg ends with row (cg & 3)'s sum
        float y[R];
        const bool b1 = cg & 2, b0 = cg & 1;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            // lanes xor 2 swap row pairs: keep rows {0,1} (b1 = 0) or {2,3} (b1 = 1)
            const float k0 = b1 ? acc[2][c] : acc[0][c], k1 = b1 ? acc[3][c] : acc[1][c];
            const float s0 = b1 ? acc[0][c] : acc[2][c], s1 = b1 ? acc[1][c] : acc[3][c];
            const float q0 = k0 + dpp_mov<0x4E>(s0), q1 = k1 + dpp_mov<0x4E>(s1);
            // lanes xor 1 swap single rows: keep row 2 b1 + b0
            float v = (b0 ? q1 : q0) + dpp_mov<0xB1>(b0 ? q0 : q1);
            v += __shfl_xor(v, 4);  // the other quad of the row group
            y[c] = v;
        }
        if (outer) {
            unsigned long long *dst = tw + (int64_t)(s & 1) * bstride + wo;
            float *pl = i >= nsw - 1 ? (((cur0 ^ (i & 1)) == 0) ? plain0 : plain1) : nullptr;
            for (int j = 0; j < rc; ++j) {
                const int64_t o = (int64_t)(port0 + rb + j) * R;
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    const float ov = 2.f * (cq[c] + y[c]) - al[(rb + j) * R + c];
                    store_word(dst + o + c, tag_word(s, ov));
                    if (pl) pl[wo + o + c] = ov;
                }
            }
        }
    }
}

// Tagged wave buffers for a persistent launch starting at sweep tag t0: buffer t0 & 1 holds the
// current waves with tag t0, the other buffer tag t0 - 1 (never the tag a reader waits for).
// ------------------------------------------------------------------ merge, residual
// Row of NR values of a row-interleaved vector (32-byte aligned for NR >= 4, 16-byte for NR = 2).
template <int NR>
__device__ inline void load_row(const double *__restrict__ p, double (&v)[NR]) {
    if constexpr (NR >= 4) {
#pragma unroll
        for (int h = 0; h < NR / 4; ++h) {
            const f64x4 t = *reinterpret_cast<const f64x4 *>(p + 4 * h);
#pragma unroll
            for (int j = 0; j < 4; ++j) v[4 * h + j] = t[j];
        }
    } else if constexpr (NR == 2) {
        const double2 t = *reinterpret_cast<const double2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    } else {
        v[0] = p[0];
    }
}

// Merged potentials (mean over the children) plus the base, written as whole rows (padding zero).
template <typename T, int R>
__global__ void k_merge(DevMaps M, int64_t nsplit, int32_t nrhs, int32_t S, const T *__restrict__ xloc,
                        const double *__restrict__ base, double *__restrict__ xout,
                        const int64_t *__restrict__ chunk_row, const int32_t *__restrict__ chunk_sys,
                        const int32_t *__restrict__ active) {
    const int ch = blockIdx.x;
    if (active && !active[chunk_sys[ch]]) return;  // a converged system keeps its x
    const int64_t v = chunk_row[ch] + threadIdx.x;
    if (v >= chunk_row[ch + 1]) return;
    const int64_t p0 = M.cp_ptr[v], p1 = M.cp_ptr[v + 1];
    const double m = (double)(p1 - p0);
    const int ng = (nrhs + R - 1) / R;
    double *xo = xout + v * S;
    const double *bo = base ? base + v * S : nullptr;
    for (int g = 0; g < ng; ++g) {
        double acc[R];
#pragma unroll
        for (int cc = 0; cc < R; ++cc) acc[cc] = 0.0;
        for (int64_t p = p0; p < p1; ++p) {
            const T *src = xloc + ((int64_t)g * nsplit + M.cp_idx[p]) * R;
#pragma unroll
            for (int cc = 0; cc < R; ++cc) acc[cc] += (double)src[cc];
        }
#pragma unroll
        for (int cc = 0; cc < R; ++cc) {
            const int c = g * R + cc;
            if (c < nrhs) xo[c] = bo ? bo[c] + acc[cc] / m : acc[cc] / m;
        }
    }
    for (int c = nrhs; c < S; ++c) xo[c] = 0.0;
}

// Sum over a wave of 64 lanes (butterfly), the result in every lane.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// r = b - A x for NR right-hand sides (block y: columns NR y .. NR y + NR - 1 of the row-interleaved
// vectors, row stride S) in one pass over A: each row's entries are read once for all of them, and x
// and b as whole rows.  One workgroup per chunk of at most 256 rows (inside one system); its entries
// are first staged in LDS by coalesced loads when they fit (else read from memory by the row's
// thread).  A chunk of a converged system (active[s] == 0) is skipped and keeps its partial sums.
constexpr int kResStage = 2560;  // matrix entries of a chunk staged in LDS (30 KiB)
template <int NR>
__global__ __launch_bounds__(kThreads) void k_residual(DevCsr A, int32_t nrhs, int32_t S, const double *__restrict__ b,
                                                       const double *__restrict__ x, double *__restrict__ r,
                                                       const int64_t *__restrict__ chunk_row,
                                                       const int32_t *__restrict__ chunk_sys,
                                                       const int32_t *__restrict__ active, int32_t nchunks,
                                                       double *__restrict__ part) {
    __shared__ int32_t scol[kResStage];
    __shared__ double sval[kResStage];
    __shared__ double red[kThreads / 64][2 * NR];
    const int ch = blockIdx.x, c0 = blockIdx.y * NR, tid = threadIdx.x;
    if (active && !active[chunk_sys[ch]]) return;
    const int64_t r0 = chunk_row[ch], r1 = chunk_row[ch + 1];
    const int64_t eb = A.rp[r0], ee = A.rp[r1];
    const bool staged = ee - eb <= kResStage;
    if (staged) {
        for (int i = tid; i < (int)(ee - eb); i += kThreads) {
            scol[i] = A.ci[eb + i];
            sval[i] = A.v[eb + i];
        }
        __syncthreads();
    }
    double rr[NR], bb[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) rr[c] = bb[c] = 0.0;
    for (int64_t v = r0 + tid; v < r1; v += kThreads) {
        double acc[NR];
        load_row<NR>(b + v * S + c0, acc);
#pragma unroll
        for (int c = 0; c < NR; ++c) bb[c] += c0 + c < nrhs ? acc[c] * acc[c] : 0.0;
        const int64_t e0 = A.rp[v], e1 = A.rp[v + 1];
        // four entries a round, their rows of x loaded together (indices past the row clamped to its
        // last entry, whose product is then weighted by zero: the loads stay unconditional)
        for (int64_t e = e0; e < e1; e += 4) {
            int32_t col[4];
            double av[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t ei = e + q < e1 ? e + q : e1 - 1;
                col[q] = staged ? scol[ei - eb] : A.ci[ei];
                const double a = staged ? sval[ei - eb] : A.v[ei];
                av[q] = e + q < e1 ? a : 0.0;
            }
            double xv[4][NR];
#pragma unroll
            for (int q = 0; q < 4; ++q) load_row<NR>(x + (int64_t)col[q] * S + c0, xv[q]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] -= av[q] * xv[q][c];
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            if (c0 + c >= nrhs) acc[c] = 0.0;  // padding columns
            rr[c] += acc[c] * acc[c];
        }
        if (r) {
            double *ro = r + v * S + c0;
#pragma unroll
            for (int c = 0; c < NR; ++c) ro[c] = acc[c];
        }
    }
    // per column: wave sums, then the four waves' partial sums added in a fixed order
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        const double sr = wave_sum(rr[c]), sb = wave_sum(bb[c]);
        if (lane == 0) {
            red[wave][2 * c] = sr;
            red[wave][2 * c + 1] = sb;
        }
    }
    __syncthreads();
    if (tid < NR && c0 + tid < nrhs) {
        double sr = 0.0, sb = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            sr += red[w][2 * tid];
            sb += red[w][2 * tid + 1];
        }
        part[((int64_t)(c0 + tid) * nchunks + ch) * 2 + 0] = sr;
        part[((int64_t)(c0 + tid) * nchunks + ch) * 2 + 1] = sb;
    }
}

// Rows of flagged systems between the two iterate (and residual) buffers, one workgroup per chunk.
__global__ void k_sys_rows(const int64_t *__restrict__ chunk_row, const int32_t *__restrict__ chunk_sys,
                           const int32_t *__restrict__ flag, int32_t S, double *__restrict__ xa,
                           double *__restrict__ xb, double *__restrict__ ra, const double *__restrict__ rb) {
    const int ch = blockIdx.x;
    const int f = flag[chunk_sys[ch]];
    if (f == 0) return;
    const int64_t lo = chunk_row[ch] * S, hi = chunk_row[ch + 1] * S;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        if (f == 3) xb[i] = xa[i];
        else xa[i] = xb[i];
        if (f == 2) ra[i] = rb[i];
    }
}

// Column-major n x nrhs (leading dimension ld) to row-interleaved rows of stride S (padding zero), and back.
__global__ void k_to_rows(const double *__restrict__ src, int64_t ld, int64_t n, int32_t nrhs, int32_t S,
                          double *__restrict__ dst) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    for (int c = 0; c < S; ++c) dst[v * S + c] = c < nrhs ? src[v + (int64_t)c * ld] : 0.0;
}

__global__ void k_from_rows(const double *__restrict__ src, int32_t S, int64_t n, int32_t nrhs,
                            double *__restrict__ dst, int64_t ld) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    for (int c = 0; c < nrhs; ++c) dst[v + (int64_t)c * ld] = src[v * S + c];
}

__global__ __launch_bounds__(256) void k_relres(const double *__restrict__ part, int32_t nchunks,
                                                 const int32_t *__restrict__ sys_chunk_ptr, int32_t nsys, int32_t nrhs,
                                                 const int32_t *__restrict__ flag, double *__restrict__ relres) {
    __shared__ double red[2][256];
    const int c = blockIdx.x / nsys, s = blockIdx.x - c * nsys, tid = threadIdx.x;
    double rr = 0.0, bb = 0.0;
    for (int q = sys_chunk_ptr[s] + tid; q < sys_chunk_ptr[s + 1]; q += 256) {
        rr += part[((int64_t)c * nchunks + q) * 2 + 0];
        bb += part[((int64_t)c * nchunks + q) * 2 + 1];
    }
    red[0][tid] = rr;
    red[1][tid] = bb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) { red[0][tid] += red[0][tid + w]; red[1][tid] += red[1][tid + w]; }
        __syncthreads();
    }
    if (tid == 0) relres[c * nsys + s] = red[1][0] > 0.0 ? sqrt(red[0][0]) / sqrt(red[1][0]) : sqrt(red[0][0]);
    if (blockIdx.x == 0 && tid == 0) relres[nsys * nrhs] = flag && *flag ? 1.0 : 0.0;  // travels with the norms
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_invz(const double *z_vtl, const int32_t *port_vtl, double *invz64, float *invz32, int64_t nports,
                 hipStream_t st) {
    if (nports == 0) return;
    hipLaunchKernelGGL(k_invz, dim3(blocks_for(nports, 256)), dim3(256), 0, st, z_vtl, port_vtl, invz64, invz32, nports);
}

void launch_factor(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_front, const double *aval,
                   const double *invz, double *vals, float *vals32, double *ws, int32_t *status,
                   const DevGreen &Gp, const int64_t *goff, double *G, hipStream_t st) {
    // 40 KiB of fronts per workgroup keeps four workgroups on a CU.  Larger fronts get the room they
    // need, up to the CU's LDS, only when every workgroup is resident even at one per CU; otherwise
    // they stay in the workspace and the CUs keep four subgraphs each in flight
    int lds_doubles = kFactorLds;
    const int need = max_front * max_front + pivot_len(max_front, true);
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
    if (need > lds_doubles && need <= (int)((kMaxLds - 1024) / sizeof(double)) && nsub <= ncu) lds_doubles = need;
    const size_t shm = sizeof(double) * (size_t)lds_doubles;
    if (shm > 64 * 1024) (void)hipFuncSetAttribute((const void *)k_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k_factor, dim3(nsub), dim3(kThreads), shm, st, S, D, aval, invz, vals, vals32, ws, lds_doubles,
                       status, Gp, goff, G);
}

void launch_gram(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_p, const DevGreen &Gp,
                 const int64_t *goff, double *G, hipStream_t st) {
    if (nsub <= 0 || max_p <= 0) return;
    const int nb = (max_p + 15) / 16, ntile = nb * (nb + 1) / 2;
    const int gy = std::min(32, (ntile + 3) / 4);  // four blocks per workgroup and pass
    hipLaunchKernelGGL(k_gram, dim3(nsub, gy), dim3(256), 0, st, S, D, Gp, goff, G);
}

void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t st) {
    if (n == 0) return;
    unsigned nb = blocks_for(n, 256);
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(256), 0, st, src, dst, n);
}

template <typename T>
void launch_split(const DevMaps &M, int64_t nsplit, const double *b, int32_t nrhs, int32_t S, int32_t R, T *bsplit,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_split<T>, dim3(blocks_for(nsplit, 256)), dim3(256), 0, st, M, nsplit, b, nrhs, S, R, bsplit);
}

void launch_sys_rows(const int64_t *chunk_row, const int32_t *chunk_sys, int32_t nchunks, const int32_t *flag,
                     int32_t S, double *xa, double *xb, double *ra, const double *rb, hipStream_t st) {
    if (nchunks > 0)
        hipLaunchKernelGGL(k_sys_rows, dim3(nchunks), dim3(256), 0, st, chunk_row, chunk_sys, flag, S, xa, xb, ra, rb);
}

void launch_to_rows(const double *src, int64_t ld, int64_t n, int32_t nrhs, int32_t S, double *dst, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_to_rows, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, ld, n, nrhs, S, dst);
}

void launch_from_rows(const double *src, int32_t S, int64_t n, int32_t nrhs, double *dst, int64_t ld, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_from_rows, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, S, n, nrhs, dst, ld);
}

template <typename T>
void launch_restart(const DevSub &D, const DevMaps &M, int32_t nsub, int32_t nlist, int64_t nsplit, int64_t nports,
                    const double *b, int32_t nrhs, int32_t S, int32_t R, T *bsplit, T *o, hipStream_t st) {
    if (nlist <= 0) return;
    hipLaunchKernelGGL(k_restart<T>, dim3(nlist), dim3(256), 0, st, D, M, nsub, nsplit, nports, b, nrhs, S, R,
                       bsplit, o);
}

// Right-hand sides per workgroup of the substitution sweep: the largest RS <= R whose LDS is at
// most 96 KiB (two workgroups per CU), else the largest that fits the CU at all (0: none fits).
template <typename T>
static int32_t sweep_rs(int32_t max_nk, int32_t max_nu, int32_t R) {
    auto need = [&](int32_t rs) { return sizeof(T) * (size_t)rs * (2 * (size_t)max_nk + (size_t)max_nu); };
    int32_t rs = R;
    while (rs > 1 && need(rs) > 96 * 1024) rs /= 2;
    return need(rs) <= kMaxLds ? rs : 0;
}

template <typename T, int R>
static const void *sweep_fn_r(int32_t rs) {
    if constexpr (R == 1) return (const void *)k_sweep<T, 1, 1>;
    else if constexpr (R == 2) return rs == 2 ? (const void *)k_sweep<T, 2, 2> : (const void *)k_sweep<T, 2, 1>;
    else if constexpr (R == 4)
        return rs == 4 ? (const void *)k_sweep<T, 4, 4> : rs == 2 ? (const void *)k_sweep<T, 4, 2> : (const void *)k_sweep<T, 4, 1>;
    else
        return rs == 8 ? (const void *)k_sweep<T, 8, 8> : rs == 4 ? (const void *)k_sweep<T, 8, 4>
             : rs == 2 ? (const void *)k_sweep<T, 8, 2> : (const void *)k_sweep<T, 8, 1>;
}
template <typename T>
static const void *sweep_fn(int32_t R, int32_t rs) {
    return R == 1 ? sweep_fn_r<T, 1>(rs) : R == 2 ? sweep_fn_r<T, 2>(rs) : R == 4 ? sweep_fn_r<T, 4>(rs) : sweep_fn_r<T, 8>(rs);
}

template <typename T>
size_t sweep_shm(int32_t max_nk, int32_t max_nu, int32_t, int32_t R) {
    const int32_t rs = sweep_rs<T>(max_nk, max_nu, R);
    return sizeof(T) * (size_t)(rs ? rs : 1) * (2 * (size_t)max_nk + (size_t)max_nu);
}

size_t sweep_lds_min(size_t tsize, int32_t max_nk, int32_t max_nu) {
    return tsize * (2 * (size_t)max_nk + (size_t)max_nu);
}

template <typename T>
hipError_t prepare_sweep(int32_t max_nk, int32_t max_nu, int32_t variant, int32_t R) {
    const int32_t rs = sweep_rs<T>(max_nk, max_nu, R);
    if (!rs) return hipErrorInvalidValue;  // a subgraph too large for the CU's LDS
    const size_t shm = sweep_shm<T>(max_nk, max_nu, variant, R);
    if (shm <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(sweep_fn<T>(R, rs), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <typename T>
void launch_sweep(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_nk, int32_t max_nu, int32_t variant,
                  int32_t ngroups, int32_t R, int32_t threads, int64_t nsplit, int64_t nports, const T *vals,
                  const T *bsplit, const int32_t *twin, const T *invz, const T *o_prev, T *o_next, T *xloc,
                  T *yout, int flags, hipStream_t st) {
    const int32_t rs = sweep_rs<T>(max_nk, max_nu, R);
    if (!rs) return;  // prepare_sweep reported it
    const size_t shm = sweep_shm<T>(max_nk, max_nu, variant, R);
    const dim3 grid(nsub, ngroups * (R / rs)), block(threads);
    void *args[] = {(void *)&S, (void *)&D, &nsplit, &nports, &vals, &bsplit, &twin, &invz, &o_prev, &o_next,
                    &xloc, &yout, &flags};
    (void)hipLaunchKernel(sweep_fn<T>(R, rs), grid, block, args, shm, st);
}

template <typename T>
static const void *ysolve_fn(int32_t R) {
    return R == 1 ? (const void *)k_ysolve<T, 1> : R == 2 ? (const void *)k_ysolve<T, 2>
         : R == 4 ? (const void *)k_ysolve<T, 4> : (const void *)k_ysolve<T, 8>;
}

template <typename T>
size_t ysolve_shm(int32_t max_nk, int32_t max_p, int32_t R) {
    return sizeof(T) * (size_t)R * (2 * (size_t)max_nk + (size_t)max_p);
}

template <typename T>
hipError_t prepare_ysolve(int32_t max_nk, int32_t max_p, int32_t R) {
    const size_t shm = ysolve_shm<T>(max_nk, max_p, R);
    if (shm > kMaxLds) return hipErrorInvalidValue;
    if (shm <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(ysolve_fn<T>(R), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <typename T>
void launch_ysolve(const DevSym &S, const DevSub &D, const DevGreen &Gp, const T *Yw, int32_t nsub, int32_t max_nk,
                   int32_t max_p, int32_t ngroups, int32_t R, int32_t threads, int64_t nsplit, int64_t nports,
                   const T *vals, const T *yb, const int32_t *twin, const T *invz, const T *o_in, T *xloc,
                   hipStream_t st) {
    const size_t shm = ysolve_shm<T>(max_nk, max_p, R);
    const dim3 grid(nsub, ngroups), block(threads);
    switch (R) {
        case 1: hipLaunchKernelGGL((k_ysolve<T, 1>), grid, block, shm, st, S, D, Gp, Yw, nsplit, nports, vals, yb, twin, invz, o_in, xloc); break;
        case 2: hipLaunchKernelGGL((k_ysolve<T, 2>), grid, block, shm, st, S, D, Gp, Yw, nsplit, nports, vals, yb, twin, invz, o_in, xloc); break;
        case 4: hipLaunchKernelGGL((k_ysolve<T, 4>), grid, block, shm, st, S, D, Gp, Yw, nsplit, nports, vals, yb, twin, invz, o_in, xloc); break;
        default: hipLaunchKernelGGL((k_ysolve<T, 8>), grid, block, shm, st, S, D, Gp, Yw, nsplit, nports, vals, yb, twin, invz, o_in, xloc); break;
    }
}

void launch_green(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_nk, int32_t max_nu, int32_t max_p,
                  const double *vals, const int64_t *goff, double *G, hipStream_t st) {
    // four port columns per workgroup when their LDS fits the CU, else one
    const size_t per = sizeof(double) * (2 * (size_t)max_nk + (size_t)max_nu);
    const int R = 4 * per <= kMaxLds ? 4 : 1;
    const size_t shm = R * per;
    const void *fn = R == 4 ? (const void *)k_green<4> : (const void *)k_green<1>;
    if (shm > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    const dim3 grid(nsub, (max_p + R - 1) / R);
    if (R == 4) hipLaunchKernelGGL(k_green<4>, grid, dim3(256), shm, st, S, D, vals, goff, G);
    else hipLaunchKernelGGL(k_green<1>, grid, dim3(256), shm, st, S, D, vals, goff, G);
}

void launch_gdiag(const DevSub &D, int32_t nsub, const int64_t *goff, const double *G, double *gd, hipStream_t st) {
    hipLaunchKernelGGL(k_gdiag, dim3(nsub), dim3(128), 0, st, D, goff, G, gd);
}

void launch_rin(const DevSub &D, int32_t nsub, const int64_t *goff, const double *G, const double *invz, double *r,
                hipStream_t st) {
    hipLaunchKernelGGL(k_rin, dim3(nsub), dim3(128), 0, st, D, goff, G, invz, r);
}

// Scratch of the allocation-free entry points: one array per GPU, held until the process ends.
// Host code never passes the name itself to a kernel (on the host it only stands for the symbol);
// it takes each device's address with hipGetSymbolAddress, once per device with that device current.
static __device__ __align__(256) double scratch[kNoAllocDoubles];

hipError_t noalloc_scratch(int device, double **ptr) {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current first
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double *>(p);
    }
    *ptr = addr[device];
    return hipSuccess;
}

template <typename T>
void launch_gather_ports(const DevSub &D, int32_t nsub, int32_t ngroups, int64_t nsplit, int32_t npg, int32_t R,
                         const T *xloc, T *cport, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_ports<T>, dim3(nsub, ngroups), dim3(128), 0, st, D, nsplit, npg, R, xloc, cport);
}

// LDS of the port-reduced sweep with W waves per subgraph: Z^{-1} a [pp][R], then W copies of y
// [R][pp + 4] and 4 values per lane for the unused lanes, which hold Z^{-1} a per port [np][R] before.
static size_t schur_lds_w(size_t tsize, int32_t max_p, int32_t max_np, int32_t R, int32_t W) {
    const size_t pp = (size_t)((max_p + 15) & ~15);
    return tsize * (pp * (size_t)R + std::max((size_t)W * ((pp + 4) * (size_t)R + 256), (size_t)max_np * R));
}

// Two waves per subgraph when one wave's LDS would leave fewer than two waves per SIMD (W = 0).
int32_t schur_waves(size_t tsize, int32_t max_p, int32_t max_np, int32_t R, int32_t W) {
    if (W == 1 || W == 2) return W;
    return schur_lds_w(tsize, max_p, max_np, R, 1) > 20 * 1024 && schur_lds_w(tsize, max_p, max_np, R, 2) <= kMaxLds ? 2 : 1;
}

size_t schur_lds_bytes(size_t tsize, int32_t max_p, int32_t max_np, int32_t R, int32_t W) {
    return schur_lds_w(tsize, max_p, max_np, R, schur_waves(tsize, max_p, max_np, R, W));
}

// One-wave teams per workgroup of the streaming sweep: four when their LDS fits the CU (a CU holds a
// limited number of workgroups, and one-wave workgroups would leave most of its wave slots empty),
// else one; teams of two waves take a workgroup each.
int schur_teams(int32_t W, size_t team_lds) {
    if (W != 1) return 1;
    const size_t tb = (team_lds + 15) & ~(size_t)15;
    return tb * 4 <= kMaxLds ? 4 : tb * 2 <= kMaxLds ? 2 : 1;
}

template <typename T, int W>
static const void *schur_fn(int32_t R) {
    return R == 1 ? (const void *)k_schur<T, 1, W> : R == 2 ? (const void *)k_schur<T, 2, W>
         : R == 4 ? (const void *)k_schur<T, 4, W> : (const void *)k_schur<T, 8, W>;
}

template <typename T>
hipError_t prepare_schur(int32_t max_p, int32_t max_np, int32_t R, int32_t W) {
    const size_t shm = schur_lds_bytes(sizeof(T), max_p, max_np, R, W);
    const int w = schur_waves(sizeof(T), max_p, max_np, R, W);
    const size_t lds = ((shm + 15) & ~(size_t)15) * schur_teams(w, shm);
    if (lds <= 64 * 1024) return hipSuccess;
    const void *fn = w == 2 ? schur_fn<T, 2>(R) : schur_fn<T, 1>(R);
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int W>
static void launch_schur_w(const DevSub &D, int32_t nsub, int32_t ngroups, int32_t R, size_t shm, int32_t npg,
                           int64_t nports, const T *G, const int64_t *goff, const T *cport, const int32_t *twin,
                           const T *invz, const T *o_prev, T *o_next, hipStream_t st) {
    const int tb = (int)((shm + 15) & ~(size_t)15);
    const int teams = schur_teams(W, shm);
    const dim3 grid((nsub + teams - 1) / teams, ngroups), block(64 * W * teams);
    const size_t lds = (size_t)tb * teams;
    switch (R) {
        case 1: hipLaunchKernelGGL((k_schur<T, 1, W>), grid, block, lds, st, D, nsub, tb, npg, nports, G, goff, cport, twin, invz, o_prev, o_next); break;
        case 2: hipLaunchKernelGGL((k_schur<T, 2, W>), grid, block, lds, st, D, nsub, tb, npg, nports, G, goff, cport, twin, invz, o_prev, o_next); break;
        case 4: hipLaunchKernelGGL((k_schur<T, 4, W>), grid, block, lds, st, D, nsub, tb, npg, nports, G, goff, cport, twin, invz, o_prev, o_next); break;
        default: hipLaunchKernelGGL((k_schur<T, 8, W>), grid, block, lds, st, D, nsub, tb, npg, nports, G, goff, cport, twin, invz, o_prev, o_next); break;
    }
}

template <typename T>
void launch_schur(const DevSub &D, int32_t nsub, int32_t ngroups, int32_t R, int32_t W, int32_t max_p, int32_t max_np,
                  int32_t npg, int64_t nports, const T *G, const int64_t *goff, const T *cport, const int32_t *twin,
                  const T *invz, const T *o_prev, T *o_next, hipStream_t st) {
    const size_t shm = schur_lds_bytes(sizeof(T), max_p, max_np, R, W);
    if (schur_waves(sizeof(T), max_p, max_np, R, W) == 2)
        launch_schur_w<T, 2>(D, nsub, ngroups, R, shm, npg, nports, G, goff, cport, twin, invz, o_prev, o_next, st);
    else
        launch_schur_w<T, 1>(D, nsub, ngroups, R, shm, npg, nports, G, goff, cport, twin, invz, o_prev, o_next, st);
}

static const void *persist_fn(int32_t R) {
    return R == 1 ? (const void *)k_schur_persist<1> : R == 2 ? (const void *)k_schur_persist<2>
         : R == 4 ? (const void *)k_schur_persist<4> : (const void *)k_schur_persist<8>;
}

size_t persist_lds_bytes(int32_t, int32_t max_np, int32_t R) {
    return sizeof(float) * ((size_t)R * (2 * 128 + 2 * (size_t)max_np) + 2 * (size_t)max_np);
}

int persist_max_p() { return 128; }

hipError_t persist_capacity(int32_t max_p, int32_t max_np, int32_t R, int64_t *resident) {
    const size_t shm = persist_lds_bytes(max_p, max_np, R);
    const void *fn = persist_fn(R);
    if (shm > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0, dev = 0, ncu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, shm);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    *resident = (int64_t)per_cu * ncu;
    return hipSuccess;
}

hipError_t launch_schur_persist(const DevSub &D, int32_t nsub, int32_t ngroups, int32_t R, int32_t max_p,
                                int32_t max_np, int32_t npg, int64_t nports, const float *G, const int64_t *goff,
                                const float *cport, const int32_t *twin, const float *invz, unsigned long long *tw,
                                float *plain0, float *plain1, int32_t t0, int32_t nsw, int32_t cur0,
                                int32_t spin_limit, int32_t *abort_flag, hipStream_t st) {
    const size_t shm = persist_lds_bytes(max_p, max_np, R);
    DevSub d = D;
    d.sub_list = nullptr;  // one workgroup per subgraph: every wave of every twin is resident
    void *args[] = {&d, &npg, &nports, &max_np, &G, &goff, &cport, &twin, &invz, &tw, &plain0, &plain1,
                    &t0, &nsw, &cur0, &spin_limit, &abort_flag};
    return hipLaunchCooperativeKernel(persist_fn(R), dim3(nsub, ngroups), dim3(256), args, (unsigned)shm, st);
}

template <typename T>
void launch_merge(const DevMaps &M, int64_t nsplit, int32_t nrhs, int32_t S, int32_t R, const T *xloc, const double *base,
                  double *xout, const int64_t *chunk_row, const int32_t *chunk_sys, int32_t nchunks,
                  const int32_t *active, hipStream_t st) {
    // one workgroup per residual chunk (at most kThreads rows)
    const dim3 grid(nchunks), block(kThreads);
    switch (R) {
        case 1: hipLaunchKernelGGL((k_merge<T, 1>), grid, block, 0, st, M, nsplit, nrhs, S, xloc, base, xout, chunk_row, chunk_sys, active); break;
        case 2: hipLaunchKernelGGL((k_merge<T, 2>), grid, block, 0, st, M, nsplit, nrhs, S, xloc, base, xout, chunk_row, chunk_sys, active); break;
        case 4: hipLaunchKernelGGL((k_merge<T, 4>), grid, block, 0, st, M, nsplit, nrhs, S, xloc, base, xout, chunk_row, chunk_sys, active); break;
        default: hipLaunchKernelGGL((k_merge<T, 8>), grid, block, 0, st, M, nsplit, nrhs, S, xloc, base, xout, chunk_row, chunk_sys, active); break;
    }
}

void launch_residual(const DevCsr &A, int64_t, int32_t nrhs, int32_t S, const double *b, const double *x, double *r,
                     const int64_t *chunk_row, const int32_t *chunk_sys, const int32_t *active, int32_t nchunks,
                     const int32_t *sys_chunk_ptr, int32_t nsys, double *part, const int32_t *flag, double *relres,
                     hipStream_t st) {
    const int NR = res_group(S);
    const dim3 grid(nchunks, S / NR), block(kThreads);
    switch (NR) {
        case 1: hipLaunchKernelGGL(k_residual<1>, grid, block, 0, st, A, nrhs, S, b, x, r, chunk_row, chunk_sys, active, nchunks, part); break;
        case 2: hipLaunchKernelGGL(k_residual<2>, grid, block, 0, st, A, nrhs, S, b, x, r, chunk_row, chunk_sys, active, nchunks, part); break;
        case 4: hipLaunchKernelGGL(k_residual<4>, grid, block, 0, st, A, nrhs, S, b, x, r, chunk_row, chunk_sys, active, nchunks, part); break;
        default: hipLaunchKernelGGL(k_residual<8>, grid, block, 0, st, A, nrhs, S, b, x, r, chunk_row, chunk_sys, active, nchunks, part); break;
    }
    hipLaunchKernelGGL(k_relres, dim3(nsys * nrhs), dim3(256), 0, st, part, nchunks, sys_chunk_ptr, nsys, nrhs, flag,
                       relres);
}

template void launch_split<double>(const DevMaps &, int64_t, const double *, int32_t, int32_t, int32_t, double *, hipStream_t);
template void launch_split<float>(const DevMaps &, int64_t, const double *, int32_t, int32_t, int32_t, float *, hipStream_t);
template void launch_restart<double>(const DevSub &, const DevMaps &, int32_t, int32_t, int64_t, int64_t, const double *, int32_t,
                                     int32_t, int32_t, double *, double *, hipStream_t);
template void launch_restart<float>(const DevSub &, const DevMaps &, int32_t, int32_t, int64_t, int64_t, const double *, int32_t,
                                    int32_t, int32_t, float *, float *, hipStream_t);
template void launch_sweep<double>(const DevSym &, const DevSub &, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t,
                                   int32_t, int64_t, int64_t, const double *, const double *, const int32_t *,
                                   const double *, const double *, double *, double *, double *, int, hipStream_t);
template void launch_sweep<float>(const DevSym &, const DevSub &, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t,
                                  int32_t, int64_t, int64_t, const float *, const float *, const int32_t *,
                                  const float *, const float *, float *, float *, float *, int, hipStream_t);
template hipError_t prepare_ysolve<double>(int32_t, int32_t, int32_t);
template hipError_t prepare_ysolve<float>(int32_t, int32_t, int32_t);
template void launch_ysolve<double>(const DevSym &, const DevSub &, const DevGreen &, const double *, int32_t, int32_t,
                                    int32_t, int32_t, int32_t, int32_t, int64_t, int64_t, const double *, const double *,
                                    const int32_t *, const double *, const double *, double *, hipStream_t);
template void launch_ysolve<float>(const DevSym &, const DevSub &, const DevGreen &, const float *, int32_t, int32_t,
                                   int32_t, int32_t, int32_t, int32_t, int64_t, int64_t, const float *, const float *,
                                   const int32_t *, const float *, const float *, float *, hipStream_t);
template hipError_t prepare_sweep<double>(int32_t, int32_t, int32_t, int32_t);
template void launch_gather_ports<double>(const DevSub &, int32_t, int32_t, int64_t, int32_t, int32_t, const double *,
                                          double *, hipStream_t);
template void launch_gather_ports<float>(const DevSub &, int32_t, int32_t, int64_t, int32_t, int32_t, const float *,
                                         float *, hipStream_t);
template hipError_t prepare_schur<double>(int32_t, int32_t, int32_t, int32_t);
template hipError_t prepare_schur<float>(int32_t, int32_t, int32_t, int32_t);
template void launch_schur<double>(const DevSub &, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, int64_t, const double *,
                                   const int64_t *, const double *, const int32_t *, const double *, const double *,
                                   double *, hipStream_t);
template void launch_schur<float>(const DevSub &, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, int64_t, const float *,
                                  const int64_t *, const float *, const int32_t *, const float *, const float *,
                                  float *, hipStream_t);
template hipError_t prepare_sweep<float>(int32_t, int32_t, int32_t, int32_t);
template void launch_merge<double>(const DevMaps &, int64_t, int32_t, int32_t, int32_t, const double *, const double *,
                                   double *, const int64_t *, const int32_t *, int32_t, const int32_t *, hipStream_t);
template void launch_merge<float>(const DevMaps &, int64_t, int32_t, int32_t, int32_t, const float *, const double *,
                                  double *, const int64_t *, const int32_t *, int32_t, const int32_t *, hipStream_t);

}  // namespace vtm
