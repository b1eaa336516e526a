/*
 * qlsd_sample.h -- the library's code-capacity noise sampler (part of libqlsd.so).
 *
 * Errors are i.i.d. Bernoulli(p_j) per fault (the code-capacity setting of Appendix D) and the
 * syndrome is s = H e over GF(2) (Sec. 2.1).  Uniforms come from the counter-based generator
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11), drawn in blocks of 4096 shots: shot g uses key (seed, g / 4096), and its fault j takes
 * 64-bit output number q = (g mod 4096) * n + j of that key, i.e. word q mod 4 of the block for
 * counter (q / 4 + 1, 0, 0, 0); u = (word >> 11) * 2^-53 and e_j = [u < p_j] (float64).  Any
 * shot range is therefore reproducible on its own, and the stream is the same as a host
 * Philox4x64-10 generator with that key and counter convention (numpy's Philox bit generator
 * with key = [seed, block] and .random()).
 *
 * Conventions as in qlsd.h: statuses, thread-local qlsd_last_error(), caller-owned device
 * buffers, asynchronous calls on `stream` (a hipStream_t as void*).
 */
#ifndef QLSD_SAMPLE_H
#define QLSD_SAMPLE_H

#include "qlsd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qlsd_sampler_s *qlsd_sampler; /* priors and logicals on the device; library-owned */

/* priors: host double[n], each in (0, 1) (QLSD_E_PRIOR otherwise).  Logical operators (nullable
 * when k = 0) as CSR over faults, host: l_row_ptr[k+1], l_col_idx[...]; a residual r fails iff
 * some row has odd overlap with r, or, with k = 0, iff r != 0 (word error).  Allocates device
 * copies; the code must outlive the sampler. */
qlsd_status qlsd_sampler_create(qlsd_code code, const double *priors, int32_t k, const int32_t *l_row_ptr,
                                const int32_t *l_col_idx, qlsd_sampler *out);

/* Shots start .. start+B-1 of stream `seed`: errors device u8[B*n] (0/1) and syndromes device
 * u8[B*m] = H e (nullable).  start >= 0, B >= 0. */
qlsd_status qlsd_sample(qlsd_sampler smp, uint64_t seed, int64_t start, int32_t B, uint8_t *errors,
                        uint8_t *syndromes, void *stream);

/* syndromes device u8[B*m] = H x for x device u8[B*n] (e.g. to check H e_hat = s). */
qlsd_status qlsd_syndromes(qlsd_sampler smp, const uint8_t *x, int32_t B, uint8_t *syndromes, void *stream);

/* fail device u8[B]: 1 iff the residual errors ^ corrections is a logical failure (see create). */
qlsd_status qlsd_failures(qlsd_sampler smp, const uint8_t *errors, const uint8_t *corrections, int32_t B,
                          uint8_t *fail, void *stream);

void qlsd_sampler_destroy(qlsd_sampler smp);

#ifdef __cplusplus
}
#endif
#endif /* QLSD_SAMPLE_H */
