/*
 * slprobe.h: C ABI of libslprobe, the benchmark's calibration library.  It
 * is not an operation of the layout method and not part of libsorlayout: it
 * measures the rates this device sustains, so that the benchmark can report
 * the force pass against what the hardware issues as well as against its
 * data-sheet peak.
 */
#ifndef SLPROBE_H
#define SLPROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The rate at which the current device issues one instruction kind:
 *   kind 0: FP32 FMA (built without packed FP32: the attainable vector FP32
 *           rate; an FMA is 2 flops)
 *   kind 1, 2, 3: rsq, sqrt, rcp (the transcendentals of the force and
 *           safeguard terms)
 * One launch of 8 waves per SIMD on `stream` (a hipStream_t), each lane
 * running 8 independent chains, timed with HIP events after one untimed
 * launch.  *per_s: lane operations per second; *ms: the timed launch.
 * Allocates and frees a 2 MiB result buffer.
 * Returns 0, -1 (another kind or a NULL output, before any device call),
 * -2 (out of device memory) or -3 (another HIP failure). */
int32_t slp_probe_rate(int32_t kind, void* stream, double* per_s, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* SLPROBE_H */
