/*
 * probe.h -- measurement support of the PME library: the LDS bandwidth of the
 * GPU, the ceiling against which the LDS traffic of the spread and gather kernels
 * (their per-tile fixed-point accumulation and staged stencil data, Sec. 2.3.2 and
 * Eqs. charge_dipole_assign, forces) is reported.  Not part of the method.
 */
#ifndef PME_PROBE_MI355X_H
#define PME_PROBE_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PME_PROBE_LDS_READ   0   /* ds_read_b128, consecutive 16 bytes per lane     */
#define PME_PROBE_LDS_ATOMIC 1   /* ds_add_u64, consecutive 8-byte slots per lane    */

/* Launch `nblocks` workgroups of 256 threads on `stream`; each thread performs
 * `iters` conflict-free LDS operations of `kind` on 64 KiB of LDS, and thread 0 of
 * each workgroup writes a checksum to out[block] (device float[nblocks]) so that
 * nothing is optimised away.  Bytes moved: nblocks * 256 * iters * (16 for reads,
 * 8 for atomics).  The caller times the launch (e.g. with events on `stream`).
 * Returns PME_OK, PME_EINVAL (kind, iters < 1, nblocks < 1, out NULL) or PME_EHIP. */
int pme_lds_probe(void* stream, int32_t kind, int32_t iters, int32_t nblocks, float* out);

#ifdef __cplusplus
}
#endif
#endif /* PME_PROBE_MI355X_H */
