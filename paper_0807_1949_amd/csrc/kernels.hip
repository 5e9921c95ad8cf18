// HIP kernels of libvtm for gfx950 (CDNA4, 64-wide wavefronts).
//
//  k_factor   one workgroup per subgraph: multifrontal Cholesky of the
//             port-augmented matrix K_k of eq. (5.8), front by front in
//             level order; the diagonal block of every supernode is stored
//             inverted so that the sweep has no long sequential chains.
//  k_sweep    one workgroup per (subgraph, group of right-hand sides): one VTM
//             sweep (Table 1 steps 3-5).  Gathers the incoming waves from the
//             twins' outgoing waves of the previous sweep (the delay of (5.6)),
//             forms the right side of (5.8), runs the level-synchronous forward
//             and backward substitutions in LDS and writes the outgoing waves
//             o_p = u_p - Z w_p = 2 u_p - a_p.
//  k_split / k_merge / k_residual: source split b_v/|S(v)|, merged potentials
//             (mean over the children) and the FP64 relative residual.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace vtm {

namespace {

constexpr int kThreads = 256;
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kWriteX = 1, kNoWaves = 2, kZeroWaves = 4;

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
// Per supernode s (front F of order f = nc + m in LDS, row-major; only its lower triangle carries
// the matrix, so the strictly upper part of the leading nc x nc block and the nc x m block to its
// right serve as scratch):
//   1. assemble: local entries, the port diagonal Z^{-1}, the children's update matrices;
//   2. L11 = chol(F11) in place (one wave when nc <= kWaveChol, else the workgroup);
//   3. Linv = L11^{-1}, column j by thread j, strictly lower part stored transposed in the upper
//      triangle (Linv[i][j] at F[j][i]; the diagonal is 1 / L11[j][j]);
//   4. L21 = F21 L11^{-T}, stored transposed in the upper-right block (L21[q][t] at F[t][nc + q]);
//   5. outputs Linv and W = L21 Linv, and the update matrix F22 - L21 L21^T written straight to
//      the workspace (lower triangle); the rank-nc update runs on the FP64 matrix cores in 16 x 16
//      tiles when m >= 16.
constexpr int kWaveChol = 48;

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(kThreads) void k_factor(DevSym S, DevSub D, const double *__restrict__ aval,
                                                     const double *__restrict__ invz, double *__restrict__ vals,
                                                     double *__restrict__ ws, int lds_front,
                                                     int32_t *__restrict__ status) {
    extern __shared__ double sm[];
    const int k = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    const ClassDev C = S.cls[D.cls[k]];
    const int nk = C.nk;
    const double *A = aval + D.aval[k];
    double *V = vals + D.val[k];
    double *W = ws + D.ws[k];
    double *dplus = W + C.ws_u + (int64_t)C.max_front * C.max_front;
    const int32_t *sn_c0 = S.sn_c0 + C.o_sn, *sn_nc = S.sn_nc + C.o_sn, *sn_m = S.sn_m + C.o_sn;
    const int32_t *sn_val = S.sn_val + C.o_sn, *sn_uoff = S.sn_uoff + C.o_sn;
    const int32_t *ch_ptr = S.ch_ptr + C.o_snp, *ch_idx = S.ch_idx + C.o_chi;
    const int32_t *sc_ptr = S.sc_ptr + C.o_snp, *sc_src = S.sc_src + C.o_sc, *sc_dst = S.sc_dst + C.o_sc;
    const int32_t *sn_ridx = S.sn_ridx + C.o_sn;
    const uint16_t *rel = S.rel + C.o_ridx;

    // diagonal additions Z^{-1} of the ports, one thread per port vertex (ports in order)
    for (int i = tid; i < nk; i += nt) dplus[i] = 0.0;
    __syncthreads();
    for (int g = D.pg_ptr[k] + tid; g < D.pg_ptr[k + 1]; g += nt) {
        double s = 0.0;
        for (int j = 0; j < D.pg_cnt[g]; ++j) s += invz[D.pg_beg[g] + j];
        dplus[D.pg_pos[g]] = s;
    }
    __syncthreads();
    int bad = 0;
    for (int s = 0; s < C.nsn; ++s) {
        const int c0 = sn_c0[s], nc = sn_nc[s], m = sn_m[s], f = nc + m;
        double *F = lds_front ? sm : W + C.ws_u;
        // 1. assembly
        for (int i = tid; i < f * f; i += nt) F[i] = 0.0;
        __syncthreads();
        for (int e = sc_ptr[s] + tid; e < sc_ptr[s + 1]; e += nt) F[sc_dst[e]] = A[sc_src[e]];
        __syncthreads();
        for (int j = tid; j < nc; j += nt) F[j * f + j] += dplus[c0 + j];
        for (int q = ch_ptr[s]; q < ch_ptr[s + 1]; ++q) {  // children one at a time (they share rows)
            __syncthreads();
            const int c = ch_idx[q], mc = sn_m[c];
            const double *U = W + sn_uoff[c];
            const uint16_t *rc = rel + sn_ridx[c];
            for (int idx = tid; idx < mc * mc; idx += nt) {
                const int a = idx / mc, b = idx - a * mc;
                if (b <= a) F[rc[a] * f + rc[b]] += U[idx];
            }
        }
        __syncthreads();
        // 2. Cholesky of the diagonal block (right-looking)
        if (nc <= kWaveChol) {
            if (wv == 0) {
                for (int kk = 0; kk < nc; ++kk) {
                    double d = F[kk * f + kk];
                    if (!(d > 0.0) || !isfinite(d)) { bad = bad ? bad : s + 1; d = 1.0; }
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
                if (!(d > 0.0) || !isfinite(d)) { bad = bad ? bad : s + 1; d = 1.0; }
                const double sd = sqrt(d), rs = 1.0 / sd;
                __syncthreads();
                for (int i = kk + 1 + tid; i < nc; i += nt) F[i * f + kk] *= rs;
                if (tid == 0) F[kk * f + kk] = sd;
                __syncthreads();
                const int T = nc - kk - 1;
                for (int idx = tid; idx < T * T; idx += nt) {
                    const int i = kk + 1 + idx / T, j = kk + 1 + idx % T;
                    if (j <= i) F[i * f + j] -= F[i * f + kk] * F[j * f + kk];
                }
                __syncthreads();
            }
        }
        __syncthreads();
        // 3. Linv, column j by thread j: Linv[i][j] = -(sum_{j <= t < i} L[i][t] Linv[t][j]) / L[i][i]
        for (int j = tid; j < nc; j += nt) {
            const double djj = 1.0 / F[j * f + j];
            for (int i = j + 1; i < nc; ++i) {
                double acc = F[i * f + j] * djj;
                for (int t = j + 1; t < i; ++t) acc += F[i * f + t] * F[j * f + t];
                F[j * f + i] = -acc / F[i * f + i];
            }
        }
        __syncthreads();
        // 4. L21[q][t] = sum_{u <= t} F21[q][u] Linv[t][u]
        for (int idx = tid; idx < m * nc; idx += nt) {
            const int q = idx / nc, t = idx - q * nc;
            const double *row = F + (nc + q) * f;
            double acc = row[t] / F[t * f + t];
            for (int u = 0; u < t; ++u) acc += row[u] * F[u * f + t];
            F[t * f + nc + q] = acc;
        }
        __syncthreads();
        // 5. outputs
        double *Vs = V + sn_val[s];
        for (int idx = tid; idx < nc * nc; idx += nt) {
            const int i = idx / nc, j = idx - i * nc;
            Vs[idx] = j > i ? 0.0 : (j == i ? 1.0 / F[i * f + i] : F[j * f + i]);
        }
        for (int idx = tid; idx < m * nc; idx += nt) {  // W[q][j] = sum_{t >= j} L21[q][t] Linv[t][j]
            const int q = idx / nc, j = idx - q * nc;
            double acc = F[j * f + nc + q] / F[j * f + j];
            for (int t = j + 1; t < nc; ++t) acc += F[t * f + nc + q] * F[j * f + t];
            Vs[nc * nc + idx] = acc;
        }
        double *Us = W + sn_uoff[s];
        if (m >= 16) {
            // update = F22 - L21 L21^T on the matrix cores: wave per 16 x 16 tile (ta, tb <= ta).
            // v_mfma_f64_16x16x4: lane l supplies A[l % 16][l / 16], B[l / 16][l % 16] and holds
            // D[4 j + l / 16][l % 16]; A[a][t] = B[t][a] = L21[a][t] = F[t][nc + a].
            const int tm = (m + 15) >> 4, ntile = tm * (tm + 1) / 2;
            const int kr = lane >> 4;
            for (int it = wv; it < ntile; it += nw) {
                int ta = (int)((sqrtf(8.0f * (float)it + 1.0f) - 1.0f) * 0.5f);
                while (ta * (ta + 1) / 2 > it) --ta;
                while ((ta + 1) * (ta + 2) / 2 <= it) ++ta;
                const int tb = it - ta * (ta + 1) / 2;
                const int ra = 16 * ta + (lane & 15), rb = 16 * tb + (lane & 15);
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
                for (int t0 = 0; t0 < nc; t0 += 4) {
                    const int t = t0 + kr;
                    const double av = (t < nc && ra < m) ? F[t * f + nc + ra] : 0.0;
                    const double bv = (t < nc && rb < m) ? F[t * f + nc + rb] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int a = 16 * ta + 4 * j + kr;
                    if (a < m && rb < m && rb <= a) Us[a * m + rb] = F[(nc + a) * f + nc + rb] - acc[j];
                }
            }
        } else {
            for (int idx = tid; idx < m * m; idx += nt) {
                const int a = idx / m, b = idx - a * m;
                if (b > a) continue;
                double acc = F[(nc + a) * f + nc + b];
                for (int t = 0; t < nc; ++t) acc -= F[t * f + nc + a] * F[t * f + nc + b];
                Us[idx] = acc;
            }
        }
        __syncthreads();
    }
    if (tid == 0) status[k] = bad;
}

// ------------------------------------------------------------------------ split
template <typename T>
__global__ void k_split(DevMaps M, int64_t nsplit, const double *__restrict__ b, int32_t nrhs, int64_t ldb, int32_t R,
                        T *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nsplit) return;
    const int32_t v = M.fvtx[e];
    const double m = (double)M.fmul[e];
    const int ng = (nrhs + R - 1) / R;
    for (int g = 0; g < ng; ++g)
        for (int cc = 0; cc < R; ++cc) {
            const int c = g * R + cc;
            out[((int64_t)g * nsplit + e) * R + cc] = c < nrhs ? (T)(b[v + (int64_t)c * ldb] / m) : (T)0;
        }
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

// Forward and backward substitution of one subgraph, R right-hand sides interleaved in LDS.
// In: vec = right side.  Out: tmp = x, vec = y (forward result).  Ends with a barrier.
template <typename T, int R, int V>
__device__ void trisolve(const ClassDev &C, const DevSym &S, const T *__restrict__ Vk, T *vec, T *tmp, T *ubuf) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int32_t *lev_c0 = S.lev_c0 + C.o_lev, *lev_u = S.lev_u + C.o_lev;
    const int32_t *colrec = S.colrec + 4 * (int64_t)C.o_col;
    const int32_t *urec = S.urec + 2 * (int64_t)C.o_ridx;
    const uint16_t *ridx = S.ridx + C.o_ridx;
    const int32_t *seg_ptr = S.seg_ptr + C.o_colp, *seg_off = S.seg_off + C.o_seg;
    const uint16_t *seg_c0 = S.seg_c0 + C.o_seg, *seg_nc = S.seg_nc + C.o_seg, *seg_u = S.seg_u + C.o_seg;
    // forward substitution, one level (independent subtrees) at a time
    for (int lv = 0; lv < C.nlev; ++lv) {
        const int cb = lev_c0[lv], ce = lev_c0[lv + 1];
        for (int i = cb + tid; i < ce; i += nt) {
            T acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = vec[i * R + c];
            const int s0 = seg_ptr[i], s1 = seg_ptr[i + 1];
            if (V == 0) {
                // pull: W_d[q, :] . t_d of every descendant supernode d with R_d[q] = i
                for (int s = s0; s < s1; ++s) {
                    const T *w = Vk + seg_off[s];
                    const T *t = tmp + seg_c0[s] * R;
                    const int n = seg_nc[s];
                    for (int j = 0; j < n; ++j) {
                        const T wj = w[j];
#pragma unroll
                        for (int c = 0; c < R; ++c) acc[c] -= wj * t[j * R + c];
                    }
                }
            } else {
                for (int s = s0; s < s1; ++s) {
                    const T *u = ubuf + seg_u[s] * R;
#pragma unroll
                    for (int c = 0; c < R; ++c) acc[c] -= u[c];
                }
            }
#pragma unroll
            for (int c = 0; c < R; ++c) tmp[i * R + c] = acc[c];
        }
        __syncthreads();
        // y = Linv t for this level's columns and (variant 1) u = W t for its update entries
        const int nrow = ce - cb;
        const int nu = V == 1 ? lev_u[lv + 1] - lev_u[lv] : 0;
        for (int task = tid; task < nrow + nu; task += nt) {
            const T *l;
            const T *t;
            int n;
            T *out;
            if (task < nrow) {
                const int i = cb + task;
                const ColRec r = load_col(colrec, i);
                const int nc = lo16(r.c0nc), jj = hi16(r.jjm);
                l = Vk + r.off + jj * nc;
                t = tmp + hi16(r.c0nc) * R;
                n = jj + 1;
                out = vec + i * R;
            } else {
                const int e = lev_u[lv] + task - nrow;
                const int2 u = reinterpret_cast<const int2 *>(urec)[e];
                l = Vk + u.x;
                t = tmp + hi16(u.y) * R;
                n = lo16(u.y);
                out = ubuf + e * R;
            }
            T acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = 0;
            for (int j = 0; j < n; ++j) {
                const T lj = l[j];
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] += lj * t[j * R + c];
            }
#pragma unroll
            for (int c = 0; c < R; ++c) out[c] = acc[c];
        }
        __syncthreads();
    }
    // backward substitution, root level first: x_s = Linv^T y_s - W^T x_R  (x kept in tmp)
    for (int lv = C.nlev - 1; lv >= 0; --lv) {
        const int cb = lev_c0[lv], ce = lev_c0[lv + 1];
        for (int j = cb + tid; j < ce; j += nt) {
            const ColRec r = load_col(colrec, j);
            const int c0 = hi16(r.c0nc), nc = lo16(r.c0nc), jj = hi16(r.jjm), m = lo16(r.jjm);
            const T *lcol = Vk + r.off + jj;
            const T *wcol = Vk + r.off + nc * nc + jj;
            const uint16_t *rr = ridx + r.ridx;
            T acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = 0;
            for (int i = jj; i < nc; ++i) {
                const T li = lcol[i * nc];
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] += li * vec[(c0 + i) * R + c];
            }
            for (int q = 0; q < m; ++q) {
                const T wq = wcol[q * nc];
                const T *x = tmp + rr[q] * R;
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] -= wq * x[c];
            }
#pragma unroll
            for (int c = 0; c < R; ++c) tmp[j * R + c] = acc[c];
        }
        __syncthreads();
    }
}

// One VTM sweep.  flags: kWriteX stores the local solutions; kNoWaves leaves o_next untouched
// (a read-only solve with the current incoming waves); kZeroWaves ignores o_prev (a = 0).
template <typename T, int R, int V>
__global__ __launch_bounds__(512) void k_sweep(DevSym S, DevSub D, int64_t nsplit, int64_t nports,
                                               const T *__restrict__ vals, const T *__restrict__ bsplit,
                                               const int32_t *__restrict__ twin, const T *__restrict__ invz,
                                               const T *__restrict__ o_prev, T *__restrict__ o_next,
                                               T *__restrict__ xloc, int flags) {
    extern __shared__ char smraw[];
    const int k = blockIdx.x, g = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
    const ClassDev C = S.cls[D.cls[k]];
    const int nk = C.nk;
    T *vec = reinterpret_cast<T *>(smraw);  // right side, then y (forward result)
    T *tmp = vec + (size_t)nk * R;          // t during the forward pass, x during the backward pass
    T *ubuf = tmp + (size_t)nk * R;         // variant 1: update entries W_s t_s of every R_s row
    const T *Vk = vals + D.val[k];
    const int64_t xo = ((int64_t)g * nsplit + D.x[k]) * R;
    const T *bs = bsplit + xo;
    const int64_t wo = (int64_t)g * nports * R;
    const bool zero_waves = flags & kZeroWaves;

    // right side of (5.8): split source + Z^{-1} * incoming wave at every port
    for (int i = tid; i < nk * R; i += nt) vec[i] = bs[i];
    __syncthreads();
    const int pg0 = D.pg_ptr[k], pg1 = D.pg_ptr[k + 1];
    if (!zero_waves) {
        for (int q = pg0 + tid; q < pg1; q += nt) {
            const int pos = D.pg_pos[q], pb = D.pg_beg[q], pc = D.pg_cnt[q];
            T acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = vec[pos * R + c];
            for (int j = 0; j < pc; ++j) {
                const T iz = invz[pb + j];
                const T *a = o_prev + wo + (int64_t)twin[pb + j] * R;
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] += a[c] * iz;
            }
#pragma unroll
            for (int c = 0; c < R; ++c) vec[pos * R + c] = acc[c];
        }
    }
    __syncthreads();
    trisolve<T, R, V>(C, S, Vk, vec, tmp, ubuf);
    // outgoing waves o_p = 2 u_p - a_p
    if (!(flags & kNoWaves)) {
        for (int q = pg0 + tid; q < pg1; q += nt) {
            const int pos = D.pg_pos[q], pb = D.pg_beg[q], pc = D.pg_cnt[q];
            for (int j = 0; j < pc; ++j) {
                const T *a = o_prev + wo + (int64_t)twin[pb + j] * R;
                T *o = o_next + wo + (int64_t)(pb + j) * R;
#pragma unroll
                for (int c = 0; c < R; ++c) o[c] = (T)2 * tmp[pos * R + c] - (zero_waves ? (T)0 : a[c]);
            }
        }
    }
    if (flags & kWriteX) {
        T *xo_ = xloc + xo;
        for (int i = tid; i < nk * R; i += nt) xo_[i] = tmp[i];
    }
}

// Port Green's functions G_k = R_k K_k^{-1} R_k^T (R_k selects the port vertices), FP64:
// column j of G_k is the port part of K_k^{-1} e_{v(j)}; blockIdx.y picks RHS columns j.
template <int V>
__global__ __launch_bounds__(256) void k_green(DevSym S, DevSub D, const double *__restrict__ vals,
                                               const int64_t *__restrict__ goff, double *__restrict__ G) {
    constexpr int R = 4;
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
    trisolve<double, R, V>(C, S, vals + D.val[k], vec, tmp, ubuf);
    double *Gk = G + goff[k];
    const int ldp = (p + 3) & ~3;  // rows padded to a multiple of 4 (padding stays zero)
    for (int idx = tid; idx < R * p; idx += nt) {
        const int c = idx / p, q = idx - c * p;
        if (j0 + c < p) Gk[(int64_t)(j0 + c) * ldp + q] = tmp[D.pg_pos[pg0 + q] * R + c];
    }
}

// Largest s in [s0, s1) with pre[s] <= it (the owner of flat item it; empty supernodes never win).
__device__ inline int owner(const int32_t *__restrict__ pre, int s0, int s1, int it) {
    int lo = s0, hi = s1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Port Green's functions by multifrontal forward substitution, one workgroup per subgraph, FP64.
// With E the unit columns of the port vertices, Y = L^{-1} E and G_k = E^T K^{-1} E = Y^T Y.  Column
// j of Y is non-zero only on the supernodes above the one holding port j, so supernode s carries
// just the w_s ports below it (a contiguous range, see DevGreen).  Its front F_s is (nc + m) x w_s
// (row-major, zero on entry except the unit entries of its own ports and what the children pushed)
// and Y_s (nc x w_s) follows it in the workspace.  Level by level:
//   phase 1  Y_s = Linv_s T_s (T_s = first nc rows of F_s); the update F_s[nc:] - W_s T_s goes into
//            the parent's front (rows by rel, columns shifted by the range offset; siblings own
//            disjoint columns, so these are plain stores);
//   phase 2  G[ports of s, ports of s] += Y_s^T Y_s (siblings own disjoint blocks of G), a
//            symmetric rank-nc update done by FP64 MFMA, 16 x 16 tiles of the lower triangle.
// Work items (phase 1) and tiles (phase 2) of a level are numbered across its supernodes through
// the prefixes py / pq.
__global__ __launch_bounds__(256) void k_green_mf(DevSym S, DevSub D, DevGreen Gp, const double *__restrict__ vals,
                                                  const int64_t *__restrict__ goff, double *__restrict__ G) {
    const int k = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    const int pg0 = D.pg_ptr[k], p = D.pg_ptr[k + 1] - pg0;
    if (p == 0) return;
    const ClassDev C = S.cls[D.cls[k]];
    const int32_t *sn_nc = S.sn_nc + C.o_sn, *sn_m = S.sn_m + C.o_sn, *sn_val = S.sn_val + C.o_sn;
    const int32_t *sn_ridx = S.sn_ridx + C.o_sn;
    const int32_t *col_sn = S.col_sn + C.o_col, *lev_c0 = S.lev_c0 + C.o_lev;
    const uint16_t *rel = S.rel + C.o_ridx;
    const int b0 = Gp.base[k];
    const int4 *pl = Gp.sn + b0;
    const int32_t *py = Gp.py + b0, *pq = Gp.pq + b0;
    const uint16_t *perm = Gp.perm + pg0;
    double *ws = Gp.ws + Gp.wso[k];
    const double *Vk = vals + D.val[k];
    double *Gk = G + goff[k];
    const int ldp = (p + 3) & ~3;
    for (int a = tid; a < p; a += nt) ws[Gp.idoff[pg0 + a]] = 1.0;
    __syncthreads();
    for (int lv = 0; lv < C.nlev; ++lv) {
        const int s0 = col_sn[lev_c0[lv]], s1 = lv + 1 < C.nlev ? col_sn[lev_c0[lv + 1]] : C.nsn;
        for (int it = py[s0] + tid; it < py[s1]; it += nt) {
            const int s = owner(py, s0, s1, it);
            const int4 e = pl[s];
            const int w = (int)((uint32_t)e.y >> 16), pc0 = e.y & 0xFFFF;
            const int nc = sn_nc[s], m = sn_m[s];
            const int loc = it - py[s], i = loc / w, a = loc - i * w;
            const double *F = ws + e.x;
            const double *V = Vk + sn_val[s];
            if (i < nc) {
                double acc = 0.0;
                for (int t = 0; t <= i; ++t) acc += V[i * nc + t] * F[t * w + a];
                ws[e.x + (nc + m) * w + i * w + a] = acc;
            } else {
                const int q = i - nc;
                const double *Wq = V + nc * nc + q * nc;
                double acc = F[i * w + a];
                for (int t = 0; t < nc; ++t) acc -= Wq[t] * F[t * w + a];
                const int pw = (int)((uint32_t)e.w >> 16), ppc0 = e.w & 0xFFFF;
                ws[e.z + (int)rel[sn_ridx[s] + q] * pw + a + (pc0 - ppc0)] = acc;
            }
        }
        __syncthreads();
        // phase 2 on the FP64 matrix cores: one wave per 16 x 16 tile (ta, tb <= ta) of Y_s^T Y_s.
        // v_mfma_f64_16x16x4: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
        // D[4 j + l / 16][l % 16] in acc[j]; here A[a][i] = Y[i][a], B[i][b] = Y[i][b].
        for (int it = pq[s0] + wv; it < pq[s1]; it += nw) {
            const int s = owner(pq, s0, s1, it);
            const int4 e = pl[s];
            const int w = (int)((uint32_t)e.y >> 16), pc0 = e.y & 0xFFFF;
            const int nc = sn_nc[s], m = sn_m[s];
            const int loc = it - pq[s];
            int ta = (int)((sqrtf(8.0f * (float)loc + 1.0f) - 1.0f) * 0.5f);
            while (ta * (ta + 1) / 2 > loc) --ta;
            while ((ta + 1) * (ta + 2) / 2 <= loc) ++ta;
            const int tb = loc - ta * (ta + 1) / 2;
            const double *Y = ws + e.x + (nc + m) * w;
            const int ra = 16 * ta + (lane & 15), rb = 16 * tb + (lane & 15), kr = lane >> 4;
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int i0 = 0; i0 < nc; i0 += 4) {
                const int i = i0 + kr;
                const double av = (i < nc && ra < w) ? Y[i * w + ra] : 0.0;
                const double bv = (i < nc && rb < w) ? Y[i * w + rb] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
            const int b = rb;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int a = 16 * ta + 4 * j + kr;
                if (a < w && b < w && (ta != tb || b <= a)) {
                    const int ja = perm[pc0 + a], jb = perm[pc0 + b];
                    Gk[(int64_t)ja * ldp + jb] += acc[j];
                    if (a != b) Gk[(int64_t)jb * ldp + ja] += acc[j];
                }
            }
        }
        // the next level's phase-1 barrier orders these G updates before the parents' ones
    }
}

// c[g][q][c] = K^{-1} b~ at the port vertices (local solutions of a zero-wave solve).
template <typename T>
__global__ void k_gather_ports(DevSub D, int64_t nsplit, int32_t npg, int32_t R, const T *__restrict__ xloc,
                               T *__restrict__ cport) {
    const int k = blockIdx.x, g = blockIdx.y;
    const int pg0 = D.pg_ptr[k], pg1 = D.pg_ptr[k + 1];
    const int64_t xo = ((int64_t)g * nsplit + D.x[k]) * R;
    for (int idx = threadIdx.x; idx < (pg1 - pg0) * R; idx += blockDim.x) {
        const int q = idx / R, c = idx - q * R;
        cport[((int64_t)g * npg + pg0 + q) * R + c] = xloc[xo + D.pg_pos[pg0 + q] * R + c];
    }
}

// Port-reduced sweep: u = c + G (Z^{-1} a) on the port vertices, then o_p = 2 u - a_p.
// G_k is symmetric and stored with a leading dimension ldp = p rounded up to 4 (zero padded):
// a thread owns VW consecutive port vertices and reads G[a * ldp + q .. q + VW) with one 16-byte
// load per column a; column slices of the workgroup are summed through LDS.
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int W = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int W = 2; };
template <typename T> __device__ inline T lane(const typename Vec16<T>::type &v, int i);
template <> __device__ inline float lane<float>(const float4 &v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
template <> __device__ inline double lane<double>(const double2 &v, int i) { return i == 0 ? v.x : v.y; }

template <typename T, int R>
__global__ __launch_bounds__(256) void k_schur(DevSub D, int32_t npg, int64_t nports, const T *__restrict__ G,
                                               const int64_t *__restrict__ goff, const T *__restrict__ cport,
                                               const int32_t *__restrict__ twin, const T *__restrict__ invz,
                                               const T *__restrict__ o_prev, T *__restrict__ o_next) {
    using V4 = typename Vec16<T>::type;
    constexpr int VW = Vec16<T>::W;
    extern __shared__ char smraw[];
    const int k = blockIdx.x, g = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
    const int pg0 = D.pg_ptr[k], p = D.pg_ptr[k + 1] - pg0;
    const int ldp = (p + 3) & ~3;
    const int64_t wo = (int64_t)g * nports * R;
    T *xz = reinterpret_cast<T *>(smraw);  // Z^{-1} a summed per port vertex [ldp][R]
    T *part = xz + (size_t)ldp * R;        // partial sums [ns][ldp][R]
    const T *Gk = G + goff[k];
    const int nrt = ldp / VW;                     // row threads
    const int rows_pass = nrt < nt ? nrt : nt;    // row threads per pass
    const int ns = nrt < nt ? nt / nrt : 1;       // column slices
    const int slice = (p + ns - 1) / ns;
    const int ldv = ldp / VW;
    // first pass: start streaming this thread's G columns before the waves arrive
    constexpr int PF = 16;
    V4 pre[PF];
    {
        const int rt = tid % rows_pass, sl = tid / rows_pass;
        const bool act = sl < ns && rt < nrt;
        const int a0 = sl * slice, a1 = act ? min(p, a0 + slice) : a0;
        const V4 *gp = reinterpret_cast<const V4 *>(Gk + rt * VW);
#pragma unroll
        for (int f = 0; f < PF; ++f) pre[f] = a0 + f < a1 ? gp[(int64_t)(a0 + f) * ldv] : V4{};
    }
    for (int q = tid; q < ldp; q += nt) {
        T acc[R];
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] = 0;
        if (q < p) {
            const int pb = D.pg_beg[pg0 + q], pc = D.pg_cnt[pg0 + q];
            for (int j = 0; j < pc; ++j) {
                const T iz = invz[pb + j];
                const T *a = o_prev + wo + (int64_t)twin[pb + j] * R;
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] += a[c] * iz;
            }
        }
#pragma unroll
        for (int c = 0; c < R; ++c) xz[q * R + c] = acc[c];
    }
    __syncthreads();
    for (int r0 = 0; r0 < nrt; r0 += rows_pass) {
        const int rt = r0 + tid % rows_pass, sl = tid / rows_pass;
        if (sl < ns && rt < nrt) {
            const int q = rt * VW;
            const int a0 = sl * slice, a1 = min(p, a0 + slice);
            T acc[VW][R];
#pragma unroll
            for (int v = 0; v < VW; ++v)
#pragma unroll
                for (int c = 0; c < R; ++c) acc[v][c] = 0;
            const V4 *gp = reinterpret_cast<const V4 *>(Gk + q);
            int a = a0;
            if (r0 == 0) {
#pragma unroll
                for (int f = 0; f < PF; ++f) {
                    if (a0 + f < a1) {
#pragma unroll
                        for (int v = 0; v < VW; ++v) {
                            const T gav = lane<T>(pre[f], v);
#pragma unroll
                            for (int c = 0; c < R; ++c) acc[v][c] += gav * xz[(a0 + f) * R + c];
                        }
                    }
                }
                a = min(a1, a0 + PF);
            }
#pragma unroll 8
            for (; a < a1; ++a) {
                const V4 gv = gp[(int64_t)a * ldv];
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const T gav = lane<T>(gv, v);
#pragma unroll
                    for (int c = 0; c < R; ++c) acc[v][c] += gav * xz[a * R + c];
                }
            }
#pragma unroll
            for (int v = 0; v < VW; ++v)
#pragma unroll
                for (int c = 0; c < R; ++c) part[((size_t)sl * ldp + q + v) * R + c] = acc[v][c];
        }
        __syncthreads();
        for (int qq = tid; qq < rows_pass * VW; qq += nt) {
            const int q = r0 * VW + qq;
            if (q >= p) continue;
            T u[R];
#pragma unroll
            for (int c = 0; c < R; ++c) u[c] = cport[((int64_t)g * npg + pg0 + q) * R + c];
            for (int sl = 0; sl < ns; ++sl)
#pragma unroll
                for (int c = 0; c < R; ++c) u[c] += part[((size_t)sl * ldp + q) * R + c];
            const int pb = D.pg_beg[pg0 + q], pc = D.pg_cnt[pg0 + q];
            for (int j = 0; j < pc; ++j) {
                const T *ai = o_prev + wo + (int64_t)twin[pb + j] * R;
                T *o = o_next + wo + (int64_t)(pb + j) * R;
#pragma unroll
                for (int c = 0; c < R; ++c) o[c] = (T)2 * u[c] - ai[c];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ merge, residual
template <typename T>
__global__ void k_merge(DevMaps M, int64_t n, int64_t nsplit, int32_t nrhs, int32_t R, const T *__restrict__ xloc,
                        const double *__restrict__ base, int64_t ldbase, double *__restrict__ xout, int64_t ldx) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t p0 = M.cp_ptr[v], p1 = M.cp_ptr[v + 1];
    const double m = (double)(p1 - p0);
    for (int c = 0; c < nrhs; ++c) {
        const int g = c / R, cc = c - g * R;
        double acc = 0.0;
        for (int64_t p = p0; p < p1; ++p) acc += (double)xloc[((int64_t)g * nsplit + M.cp_idx[p]) * R + cc];
        const double xb = acc / m;
        xout[v + (int64_t)c * ldx] = base ? base[v + (int64_t)c * ldbase] + xb : xb;
    }
}

__global__ __launch_bounds__(kThreads) void k_residual(DevCsr A, int32_t nrhs, const double *__restrict__ b, int64_t ldb,
                                                       const double *__restrict__ x, int64_t ldx, double *__restrict__ r,
                                                       int64_t ldr, const int64_t *__restrict__ chunk_row,
                                                       int32_t nchunks, double *__restrict__ part) {
    __shared__ double red[2][kThreads];
    const int ch = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    const int64_t r0 = chunk_row[ch], r1 = chunk_row[ch + 1];
    double rr = 0.0, bb = 0.0;
    for (int64_t v = r0 + tid; v < r1; v += kThreads) {
        const double bv = b[v + (int64_t)c * ldb];
        double acc = bv;
        for (int64_t e = A.rp[v]; e < A.rp[v + 1]; ++e) acc -= A.v[e] * x[A.ci[e] + (int64_t)c * ldx];
        if (r) r[v + (int64_t)c * ldr] = acc;
        rr += acc * acc;
        bb += bv * bv;
    }
    red[0][tid] = rr;
    red[1][tid] = bb;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (tid < s) { red[0][tid] += red[0][tid + s]; red[1][tid] += red[1][tid + s]; }
        __syncthreads();
    }
    if (tid == 0) {
        part[((int64_t)c * nchunks + ch) * 2 + 0] = red[0][0];
        part[((int64_t)c * nchunks + ch) * 2 + 1] = red[1][0];
    }
}

__global__ __launch_bounds__(256) void k_relres(const double *__restrict__ part, int32_t nchunks,
                                                 const int32_t *__restrict__ sys_chunk_ptr, int32_t nsys, int32_t nrhs,
                                                 double *__restrict__ relres) {
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
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_invz(const double *z_vtl, const int32_t *port_vtl, double *invz64, float *invz32, int64_t nports,
                 hipStream_t st) {
    if (nports == 0) return;
    hipLaunchKernelGGL(k_invz, dim3(blocks_for(nports, 256)), dim3(256), 0, st, z_vtl, port_vtl, invz64, invz32, nports);
}

void launch_factor(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_nk, int32_t max_front,
                   const double *aval, const double *invz, double *vals, double *ws, int64_t, int32_t *status,
                   hipStream_t st) {
    (void)max_nk;
    const size_t front = sizeof(double) * (size_t)max_front * max_front;
    const int lds_front = front <= 96 * 1024;
    const size_t shm = lds_front ? front : 0;
    if (shm > 64 * 1024) (void)hipFuncSetAttribute((const void *)k_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k_factor, dim3(nsub), dim3(kThreads), shm, st, S, D, aval, invz, vals, ws, lds_front, status);
}

void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t st) {
    if (n == 0) return;
    unsigned nb = blocks_for(n, 256);
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(256), 0, st, src, dst, n);
}

template <typename T>
void launch_split(const DevMaps &M, int64_t nsplit, const double *b, int32_t nrhs, int64_t ldb, int32_t R, T *bsplit,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_split<T>, dim3(blocks_for(nsplit, 256)), dim3(256), 0, st, M, nsplit, b, nrhs, ldb, R, bsplit);
}

template <typename T, int V>
static const void *sweep_fn_v(int32_t R) {
    return R == 1 ? (const void *)k_sweep<T, 1, V> : R == 2 ? (const void *)k_sweep<T, 2, V>
         : R == 4 ? (const void *)k_sweep<T, 4, V> : (const void *)k_sweep<T, 8, V>;
}

template <typename T>
size_t sweep_shm(int32_t max_nk, int32_t max_nu, int32_t variant, int32_t R) {
    return sizeof(T) * (size_t)R * (2 * (size_t)max_nk + (variant == 1 ? (size_t)max_nu : 0));
}

template <typename T>
hipError_t prepare_sweep(int32_t max_nk, int32_t max_nu, int32_t variant, int32_t R) {
    const size_t shm = sweep_shm<T>(max_nk, max_nu, variant, R);
    if (shm <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(variant == 1 ? sweep_fn_v<T, 1>(R) : sweep_fn_v<T, 0>(R),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <typename T, int V>
static void launch_sweep_v(const DevSym &S, const DevSub &D, dim3 grid, dim3 block, size_t shm, int32_t R,
                           int64_t nsplit, int64_t nports, const T *vals, const T *bsplit, const int32_t *twin,
                           const T *invz, const T *o_prev, T *o_next, T *xloc, int flags, hipStream_t st) {
    switch (R) {
        case 1: hipLaunchKernelGGL((k_sweep<T, 1, V>), grid, block, shm, st, S, D, nsplit, nports, vals, bsplit, twin, invz, o_prev, o_next, xloc, flags); break;
        case 2: hipLaunchKernelGGL((k_sweep<T, 2, V>), grid, block, shm, st, S, D, nsplit, nports, vals, bsplit, twin, invz, o_prev, o_next, xloc, flags); break;
        case 4: hipLaunchKernelGGL((k_sweep<T, 4, V>), grid, block, shm, st, S, D, nsplit, nports, vals, bsplit, twin, invz, o_prev, o_next, xloc, flags); break;
        default: hipLaunchKernelGGL((k_sweep<T, 8, V>), grid, block, shm, st, S, D, nsplit, nports, vals, bsplit, twin, invz, o_prev, o_next, xloc, flags); break;
    }
}

template <typename T>
void launch_sweep(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_nk, int32_t max_nu, int32_t variant,
                  int32_t ngroups, int32_t R, int32_t threads, int64_t nsplit, int64_t nports, const T *vals,
                  const T *bsplit, const int32_t *twin, const T *invz, const T *o_prev, T *o_next, T *xloc,
                  int flags, hipStream_t st) {
    const size_t shm = sweep_shm<T>(max_nk, max_nu, variant, R);
    const dim3 grid(nsub, ngroups), block(threads);
    if (variant == 1)
        launch_sweep_v<T, 1>(S, D, grid, block, shm, R, nsplit, nports, vals, bsplit, twin, invz, o_prev, o_next, xloc, flags, st);
    else
        launch_sweep_v<T, 0>(S, D, grid, block, shm, R, nsplit, nports, vals, bsplit, twin, invz, o_prev, o_next, xloc, flags, st);
}

void launch_green(const DevSym &S, const DevSub &D, int32_t nsub, int32_t max_nk, int32_t max_nu, int32_t max_p,
                  const double *vals, const int64_t *goff, double *G, hipStream_t st) {
    const int V = 2 * (size_t)max_nk + max_nu <= 96 * 1024 / (8 * 4) ? 1 : 0;
    const size_t shm = sizeof(double) * 4 * (2 * (size_t)max_nk + (V ? (size_t)max_nu : 0));
    const void *fn = V ? (const void *)k_green<1> : (const void *)k_green<0>;
    if (shm > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    const dim3 grid(nsub, (max_p + 3) / 4);
    if (V) hipLaunchKernelGGL(k_green<1>, grid, dim3(256), shm, st, S, D, vals, goff, G);
    else hipLaunchKernelGGL(k_green<0>, grid, dim3(256), shm, st, S, D, vals, goff, G);
}

void launch_green_mf(const DevSym &S, const DevSub &D, const DevGreen &Gp, int32_t nsub, const double *vals,
                     const int64_t *goff, double *G, hipStream_t st) {
    hipLaunchKernelGGL(k_green_mf, dim3(nsub), dim3(256), 0, st, S, D, Gp, vals, goff, G);
}

template <typename T>
void launch_gather_ports(const DevSub &D, int32_t nsub, int32_t ngroups, int64_t nsplit, int32_t npg, int32_t R,
                         const T *xloc, T *cport, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_ports<T>, dim3(nsub, ngroups), dim3(128), 0, st, D, nsplit, npg, R, xloc, cport);
}

template <typename T>
size_t schur_shm(int32_t max_p, int32_t R, int32_t threads) {
    // xz [ldp][R] + partial sums: at most (threads / row threads) slices of ldp rows <= ldp + threads * VW
    const size_t ldp = (size_t)((max_p + 3) & ~3);
    return sizeof(T) * (size_t)R * (ldp + (size_t)threads * Vec16<T>::W + ldp);
}

template <typename T>
hipError_t prepare_schur(int32_t max_p, int32_t R) {
    const size_t shm = schur_shm<T>(max_p, R, 256);
    if (shm <= 64 * 1024) return hipSuccess;
    const void *fn = R == 1 ? (const void *)k_schur<T, 1> : R == 2 ? (const void *)k_schur<T, 2>
                   : R == 4 ? (const void *)k_schur<T, 4> : (const void *)k_schur<T, 8>;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <typename T>
void launch_schur(const DevSub &D, int32_t nsub, int32_t ngroups, int32_t R, int32_t max_p, int32_t npg,
                  int64_t nports, const T *G, const int64_t *goff, const T *cport, const int32_t *twin,
                  const T *invz, const T *o_prev, T *o_next, hipStream_t st) {
    const size_t shm = schur_shm<T>(max_p, R, 256);
    const dim3 grid(nsub, ngroups), block(256);
    switch (R) {
        case 1: hipLaunchKernelGGL((k_schur<T, 1>), grid, block, shm, st, D, npg, nports, G, goff, cport, twin, invz, o_prev, o_next); break;
        case 2: hipLaunchKernelGGL((k_schur<T, 2>), grid, block, shm, st, D, npg, nports, G, goff, cport, twin, invz, o_prev, o_next); break;
        case 4: hipLaunchKernelGGL((k_schur<T, 4>), grid, block, shm, st, D, npg, nports, G, goff, cport, twin, invz, o_prev, o_next); break;
        default: hipLaunchKernelGGL((k_schur<T, 8>), grid, block, shm, st, D, npg, nports, G, goff, cport, twin, invz, o_prev, o_next); break;
    }
}

template <typename T>
void launch_merge(const DevMaps &M, int64_t n, int64_t nsplit, int32_t nrhs, int32_t R, const T *xloc,
                  const double *base, int64_t ldbase, double *xout, int64_t ldx, hipStream_t st) {
    hipLaunchKernelGGL(k_merge<T>, dim3(blocks_for(n, 256)), dim3(256), 0, st, M, n, nsplit, nrhs, R, xloc, base, ldbase,
                       xout, ldx);
}

void launch_residual(const DevCsr &A, int64_t, int32_t nrhs, const double *b, int64_t ldb, const double *x, int64_t ldx,
                     double *r, int64_t ldr, const int64_t *chunk_row, const int32_t *, int32_t nchunks,
                     const int32_t *sys_chunk_ptr, int32_t nsys, double *part, double *relres, hipStream_t st) {
    hipLaunchKernelGGL(k_residual, dim3(nchunks, nrhs), dim3(kThreads), 0, st, A, nrhs, b, ldb, x, ldx, r, ldr,
                       chunk_row, nchunks, part);
    hipLaunchKernelGGL(k_relres, dim3(nsys * nrhs), dim3(256), 0, st, part, nchunks, sys_chunk_ptr, nsys, nrhs, relres);
}

template void launch_split<double>(const DevMaps &, int64_t, const double *, int32_t, int64_t, int32_t, double *, hipStream_t);
template void launch_split<float>(const DevMaps &, int64_t, const double *, int32_t, int64_t, int32_t, float *, hipStream_t);
template void launch_sweep<double>(const DevSym &, const DevSub &, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t,
                                   int32_t, int64_t, int64_t, const double *, const double *, const int32_t *,
                                   const double *, const double *, double *, double *, int, hipStream_t);
template void launch_sweep<float>(const DevSym &, const DevSub &, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t,
                                  int32_t, int64_t, int64_t, const float *, const float *, const int32_t *,
                                  const float *, const float *, float *, float *, int, hipStream_t);
template hipError_t prepare_sweep<double>(int32_t, int32_t, int32_t, int32_t);
template void launch_gather_ports<double>(const DevSub &, int32_t, int32_t, int64_t, int32_t, int32_t, const double *,
                                          double *, hipStream_t);
template void launch_gather_ports<float>(const DevSub &, int32_t, int32_t, int64_t, int32_t, int32_t, const float *,
                                         float *, hipStream_t);
template hipError_t prepare_schur<double>(int32_t, int32_t);
template hipError_t prepare_schur<float>(int32_t, int32_t);
template void launch_schur<double>(const DevSub &, int32_t, int32_t, int32_t, int32_t, int32_t, int64_t, const double *,
                                   const int64_t *, const double *, const int32_t *, const double *, const double *,
                                   double *, hipStream_t);
template void launch_schur<float>(const DevSub &, int32_t, int32_t, int32_t, int32_t, int32_t, int64_t, const float *,
                                  const int64_t *, const float *, const int32_t *, const float *, const float *,
                                  float *, hipStream_t);
template hipError_t prepare_sweep<float>(int32_t, int32_t, int32_t, int32_t);
template void launch_merge<double>(const DevMaps &, int64_t, int64_t, int32_t, int32_t, const double *, const double *,
                                   int64_t, double *, int64_t, hipStream_t);
template void launch_merge<float>(const DevMaps &, int64_t, int64_t, int32_t, int32_t, const float *, const double *,
                                  int64_t, double *, int64_t, hipStream_t);

}  // namespace vtm
