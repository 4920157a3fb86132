/*
 * lbfast_measure.h -- measurement utilities of liblbfast.so.  They are not
 * part of the method: copy kernels of known size, used to calibrate hardware
 * traffic counters against the step and to measure the bandwidth ceiling
 * the step is set against.  Same status codes and error reporting as
 * lbfast.h.
 */
#ifndef LBFAST_MEASURE_H_
#define LBFAST_MEASURE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Measurement utility, not part of the method: copy `nplanes` planes of `n`
 * floats from src to dst (device pointers, n * 4 < 2^32) on `stream`, using
 * the same memory instruction forms as the step (dword buffer loads,
 * non-temporal dword buffer stores).  A copy of known size, used to calibrate
 * hardware traffic counters against the step. */
int lbfast_stream_probe(const void* src, void* dst, int64_t n, int nplanes, void* stream);

/* Measurement utility, not part of the method: copy n4 16-byte elements from
 * src to dst (device pointers, 16-byte aligned) on `stream`, one 16-byte
 * access per thread in a one-shot grid, non-temporal stores: the fastest
 * copy form measured on MI355X, the bandwidth ceiling of a single stream that
 * reads and writes equal volumes. */
int lbfast_copy_probe(const void* src, void* dst, int64_t n4, void* stream);

/* Measurement utility, not part of the method: copy nplanes (1..10) planes
 * of n floats (n even) in structure of arrays from src to dst (device
 * pointers, 8-byte aligned), each thread moving two consecutive floats of
 * every plane (all loads, then all non-temporal stores): the step's load and
 * store pattern without halos or arithmetic, the ceiling the step is set
 * against. */
int lbfast_planes_probe(const void* src, void* dst, int64_t n, int nplanes, void* stream);

/* Measurement utility, not part of the method: copy a state of
 * nx x ny x nz sites from src to dst (device pointers, 16-byte aligned) in
 * the step's marching order without halos or arithmetic: workgroups of
 * 128 x 8 column tiles (two sites per lane, one row per wave) march through
 * chunks of zchunk z-planes, loading plane z + 1 while storing plane z
 * (non-temporal stores).  nx a multiple of 128, ny a multiple of 8.  The
 * state holds ten moment planes in one of four layouts (bytes per site S):
 *   0  FP32, plane after plane (S = 40)
 *   1  16-bit, plane after plane (S = 20)
 *   2  16-bit, planes in pairs, one 32-bit word per site each (S = 20)
 *   3  16-bit, the library's layout: two groups of four planes (one 64-bit
 *      word per site each) and a pair (S = 20)
 * src and dst each hold S x nx x ny x nz bytes.  It sets the marching
 * step's access pattern against the layout of its 16-bit state. */
int lbfast_zmarch_probe(const void* src, void* dst, int nx, int ny, int nz, int layout,
                        int zchunk, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBFAST_MEASURE_H_ */
