/*
 * ace_probe.h — streaming bandwidth probes for the gfx950 ACE library.
 *
 * Not part of the method: these measure the HBM rates that the transform
 * passes of ace_build can reach on the device, so that each pass can be
 * reported against both the HBM peak and the rate a plain streaming kernel
 * of the same access kind attains.
 *
 * ace_bandwidth_probe: one launch over `bytes` of caller-owned device memory
 *   `buf` (16-byte aligned), `blocks` workgroups of 256 threads, each thread
 *   handling 16-byte values, four in flight, on `stream` (a hipStream_t):
 *     ACE_PROBE_READ_WRITE  read every value and write it back scaled by
 *                           1 + 1e-10 (16 B read + 16 B written per value);
 *     ACE_PROBE_READ        read every value (contents unchanged);
 *     ACE_PROBE_WRITE       write 1.0 to every double.
 *   Returns 0, 1 for a null or misaligned buffer, fewer than 16 bytes, an
 *   unknown kind or blocks outside 1 .. 2^20, or 4 when the launch fails.
 */
#ifndef ACE_PROBE_H_
#define ACE_PROBE_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACE_PROBE_READ_WRITE 0
#define ACE_PROBE_READ 1
#define ACE_PROBE_WRITE 2
int ace_bandwidth_probe(int kind, void *stream, void *buf, size_t bytes, int blocks);

#ifdef __cplusplus
}
#endif

#endif /* ACE_PROBE_H_ */
