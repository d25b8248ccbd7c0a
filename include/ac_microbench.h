/*
 * ac_microbench.h -- roofline denominators for the Aho-Corasick scan on
 * MI355X (gfx950): C ABI of libac_microbench.so.
 *
 * The scan's kernels are bound by HBM bandwidth (text in, matches out), by
 * table lookups in LDS or L2, or by the latency of one dependent lookup per
 * symbol (the single pass of section III.A).  These calls measure each of
 * those ceilings on the device with the simplest kernel that reaches it, so
 * the benchmark can state measured peaks beside the published ones.
 *
 * All pointers are device memory (hipMalloc or a torch tensor's data
 * pointer) owned by the caller.  Each call runs its kernel once to warm up,
 * then `reps` times back to back on the library's own stream, waits, and
 * returns the mean time per launch.  Calls are not thread safe.
 * Return value: ACB_OK, ACB_E_INVALID (bad argument; nothing launched) or
 * ACB_E_HIP (a HIP call failed).
 */
#ifndef AC_MICROBENCH_H
#define AC_MICROBENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACB_OK 0
#define ACB_E_INVALID (-1)
#define ACB_E_HIP (-7)

/* Copy `bytes` (multiple of 16) from d_src to d_dst with 16-byte
 * non-temporal loads and stores, one 4 KiB piece per block; moves 2 * bytes
 * of HBM traffic. */
int acb_hbm_copy(void *d_dst, const void *d_src, uint64_t bytes, int reps, double *ms);
/* Write `bytes` (multiple of 16) of d_dst with 16-byte stores, one 4 KiB
 * piece per block. */
int acb_hbm_write(void *d_dst, uint64_t bytes, int reps, double *ms);
/* Read `bytes` (multiple of 16) of d_src with 16-byte non-temporal loads,
 * one 4 KiB piece per block. */
int acb_hbm_read(const void *d_src, uint64_t bytes, int reps, double *ms);

/* ds_read_b32 throughput: one 1024-thread block per compute unit reads a
 * 64 KiB LDS table, 16 reads per lane per iteration.  random = 0: the 64
 * lanes of a wave read 64 distinct banks; random != 0: random addresses (the
 * access pattern of the scan's table lookups).  *reads = dword reads per
 * launch. */
int acb_lds_read(int random, uint32_t iters, int reps, double *ms, uint64_t *reads);

/* Random dword gathers from a device table of `entries` uint32 (a power of
 * two, 64 .. 2^31): 8 independent loads per lane per iteration.  A table of a
 * few MiB stays in L2; larger ones spill to the MALL and HBM.  *reads = loads
 * per launch. */
int acb_gather(const uint32_t *d_table, uint64_t entries, uint32_t iters, int reps, double *ms,
               uint64_t *reads);

/* Latency of dependent loads: one wave whose lane l starts at l and follows
 * d_next (which must hold a permutation of 0 .. entries-1, entries >= 64)
 * `steps` times; lds != 0 copies the table into LDS first (entries <=
 * 16384).  *ns_per_step = time per step of the chain. */
int acb_chase(const uint32_t *d_next, uint64_t entries, int lds, uint32_t steps, int reps,
              double *ns_per_step);

#ifdef __cplusplus
}
#endif
#endif /* AC_MICROBENCH_H */
