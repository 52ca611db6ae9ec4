/*
 * probe.h -- measurement support of the PME library: the LDS bandwidth of the
 * GPU, the ceiling against which the LDS traffic of the spread and gather kernels
 * (their per-tile fixed-point accumulation and staged stencil data, Sec. 2.3.2 and
 * Eqs. charge_dipole_assign, forces) is reported, and the global-memory cost of
 * combining overlapping per-tile regions, which decides the spread's design.  Not
 * part of the method.
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

/* Halo-combination probe: the global-memory cost of a "scatter-once" spread, the
 * alternative to the owner-computes tiles of the spread kernels.  In such a spread
 * each tile would add the whole stencils of its own atoms (anchors in the tile) into
 * an LDS region of R = T + p - 1 points per axis, starting (p - 1)/2 points
 * before the tile; the regions of neighbouring tiles overlap by p - 1 points, so
 * they have to be combined in global memory.  The probe moves exactly that data
 * (region words carry 1, not charges):
 *   HALO_ATOMIC  every region added into `mesh` (int64, N0 N1 N2, zeroed by the
 *                caller) with one 64-bit global atomic add per region point;
 *   HALO_WRITE   every region written contiguously into `regions` (int64, one
 *                block of R0 R1 R2 words per tile, tiles in x-major order);
 *   HALO_FOLD    the regions of HALO_WRITE summed per mesh point, in a fixed
 *                order, into `mesh` (float, N0 N1 N2): one thread per point.
 * One workgroup of 256 threads per tile (ATOMIC, WRITE) or per 256 points (FOLD),
 * on `stream`; the caller times the launch.  Needs N[a] % T[a] == 0 and
 * N[a] >= T[a] + p - 1 on every axis (each point then lies in one or two regions
 * per axis) and 1 <= p <= 8.  Returns PME_OK, PME_EINVAL (kind, sizes, NULL
 * buffer) or PME_EHIP. */
#define PME_PROBE_HALO_ATOMIC 2
#define PME_PROBE_HALO_WRITE  3
#define PME_PROBE_HALO_FOLD   4
int pme_halo_probe(void* stream, int32_t kind, const int32_t N[3], const int32_t T[3], int32_t p,
                   void* regions, void* mesh);

#ifdef __cplusplus
}
#endif
#endif /* PME_PROBE_MI355X_H */
