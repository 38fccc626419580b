/*
 * eik_probe.h -- bandwidth probes of the device the solver runs on (libeik_probe.so).
 *
 * The solver's kernels are judged against two rooflines: HBM bandwidth for the cells' global
 * traffic and LDS bandwidth for the in-cell sweeps.  The peaks (8 TB/s HBM3E; 256 CUs x 256 B
 * per clock x 2.4 GHz = 157 TB/s LDS, a figure the LDS read probe's 161 B per clock per CU
 * already shows the older 128 B per clock to understate) are what the bench reports fractions
 * of; these probes measure what plain kernels reach on the same device, so that the fractions
 * can be read against an achievable figure too.  They are measurement tools, not part of the
 * solve.
 *
 * All pointers are device pointers; the caller owns every buffer.  Every call enqueues on
 * `stream`, waits for it, and returns 0 or -3 (a HIP error) / -1 (invalid argument).
 */
#ifndef EIK_PROBE_H
#define EIK_PROBE_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * eikp_copy -- dst[0 .. bytes) <- src[0 .. bytes) with 16-byte vector loads and stores, `reps`
 * times (1..1000) after one untimed launch; *ms receives the mean duration of one copy (HIP
 * events around the timed launches).  bytes must be a positive multiple of 16 and both pointers
 * 16-byte aligned; the buffers must not overlap.  Moves 2 * bytes per copy.
 */
int eikp_copy(const void* src, void* dst, size_t bytes, int reps, hipStream_t stream, float* ms);

/*
 * eikp_lds -- LDS bandwidth: `blocks` workgroups (1..65536) of 256 threads, each with a 32 KiB
 * LDS array (four workgroups fit one CU), read it (write = 0; filled first) or write it
 * (write = 1) with 16-byte accesses, `iters` (1..2^20) per thread, bank-conflict free
 * (consecutive lanes, consecutive 16-byte words).  One untimed launch, then `reps` (1..1000)
 * timed; *ms receives the mean duration of one launch and *bytes_moved (may be NULL) the LDS
 * bytes one launch reads or writes in its timed loop (blocks * 256 * iters * 16).  out
 * (blocks * 256 uint32, device) receives a per-thread checksum so that no access is dead code:
 * for reads the XOR of the four 32-bit lanes of every word the thread read, for writes the
 * same XOR over the 8 words of the thread's column (t + 256 m) read back at the end (defined
 * when iters >= 8: iteration k writes (t + k, k, t, 1) to word t + 256 (k mod 8)).
 */
int eikp_lds(int blocks, int iters, int write, int reps, unsigned int* out, hipStream_t stream,
             float* ms, double* bytes_moved);

#ifdef __cplusplus
}
#endif

#endif /* EIK_PROBE_H */
