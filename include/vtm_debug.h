/*
 * vtm_debug.h -- introspection of libvtm's symbolic analysis, for tests.
 *
 * Not needed to solve systems.  It exposes the per-class data that the
 * device factorisation and sweep consume, so that a host test can re-run the
 * multifrontal elimination of eq. (5.8)'s local matrices from it and compare
 * with a dense factorisation.
 */
#ifndef VTM_DEBUG_H
#define VTM_DEBUG_H

#include "vtm.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Symbolic data of the class of subgraph k (after vtm_evs_partition).
 * sizes[8] = {nk, nsn, nlev, n_ridx, n_scatter, nval, ws_u, class id}; call
 * once with only sizes to size the other arrays (any may be NULL):
 *   perm[nk]        factor position -> local index (local = rank of the global id)
 *   sn[10*nsn]      per supernode {c0, nc, m, val_off, ridx_off, parent, level, u_off,
 *                   first and end of its assembly pairs}
 *   lev_c0[nlev+1]  first factor column of every level
 *   ridx[n_ridx]    off-diagonal rows R_s (factor positions) of every supernode
 *   rel[n_ridx]     position of each R_s row in the parent's front (cols then R)
 *   sc[2*n_scatter] assembly pairs {local CSR entry, row-major front position}
 * Errors: VTM_ERR_INVALID, VTM_ERR_STATE (no partition or k out of range).
 */
vtm_status vtm_debug_class(vtm_handle h, int32_t k, int64_t *sizes, int32_t *perm, int32_t *sn, int32_t *lev_c0,
                           uint16_t *ridx, uint16_t *rel, int32_t *sc);

#ifdef __cplusplus
}
#endif

#endif /* VTM_DEBUG_H */
