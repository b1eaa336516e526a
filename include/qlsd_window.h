/*
 * qlsd_window.h -- overlapping-window decoding of multi-round detector error models (part of
 * libqlsd.so).
 *
 * The (w, c) window scheme of the paper's multi-round simulations (Sec. 4.3, numerical decoding
 * simulations, w = 3, c = 1): detectors carry a syndrome round; a fault's round is the earliest
 * round among its detectors.  Windows of w rounds start at rounds 0, c, 2c, ... while a further
 * window fits, and a last window runs to the final round.  Each window decodes (BP, then LSD as
 * set in qlsd_params) the detectors of its rounds against the faults of its rounds, on the
 * syndrome left by the faults committed so far, and commits the faults of its first c rounds
 * (the last window commits all of its faults).  Every decoded window is an ordinary qlsd decoder
 * on the window's sub-matrix; all of a batch's windows run on the device, one after another,
 * without host round trips.
 *
 * Conventions as in qlsd.h.
 */
#ifndef QLSD_WINDOW_H
#define QLSD_WINDOW_H

#include "qlsd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qlsd_window_s *qlsd_window; /* window sub-codes, decoders and index maps; library-owned */

/* det_round: host int32[m], the syndrome round of each detector (>= 0); priors: host double[n];
 * 1 <= c < w.  Creates one decoder per window (params as for qlsd_decoder_create, each sized for
 * max_batch shots).  The code must outlive the window decoder. */
qlsd_status qlsd_window_create(qlsd_code code, const double *priors, const int32_t *det_round, int32_t w,
                               int32_t c, const qlsd_params *params, int32_t max_batch, qlsd_window *out);

/* syndromes device u8[B*m] (all rounds) -> corrections device u8[B*n]; 0 <= B <= max_batch.
 * Asynchronous on `stream`; the result satisfies H e = s whenever every window's decode does. */
qlsd_status qlsd_window_decode(qlsd_window wd, const uint8_t *syndromes, int32_t B, uint8_t *corrections,
                               void *stream);

/* Number of windows (steps) of the scheme. */
int32_t qlsd_window_count(qlsd_window wd);

void qlsd_window_destroy(qlsd_window wd);

#ifdef __cplusplus
}
#endif
#endif /* QLSD_WINDOW_H */
