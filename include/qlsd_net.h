/*
 * qlsd_net.h -- learned reliability refinement between BP and LSD (part of libqlsd.so).
 *
 * Not part of the paper.  LSD consumes only the *order* of its input soft information (the
 * growth step picks the candidate of lowest LLR, Sec. 4.1 step 2), so a small network over the
 * Tanner graph may re-rank BP's posteriors before LSD sees them.  With posteriors L (float32),
 * prior LLRs lambda and syndrome s of one shot, and hidden width 32:
 *
 *   x_j   = (tanh(L_j/8), lambda_j/8),   h0_j = relu(W0 x_j + b0)
 *   for l = 1..3:  m_i = mean_{j in N(i)} h_{l-1,j},   c_i = relu(A_l m_i + (1 - 2 s_i) a_l)
 *                  g_j = mean_{i in N(j)} c_i,          h_l,j = relu(B_l h_{l-1,j} + C_l g_j + b_l)
 *   Delta_j = w . h_3,j + b_out,   L'_j = L_j + Delta_j
 *
 * trained with the mean binary cross-entropy of P(e_j = 1) = sigmoid(-L'_j) against the true
 * error.  Parameters are QLSD_NET_PARAMS floats in the order W0(32x2), b0, then per layer
 * A(32x32), a, B(32x32), C(32x32), b, then w, b_out (matrices row-major, out x in).  The dense
 * products run on bf16 MFMA with float32 accumulation; sums over neighbours in float32.
 * With w = 0 and b_out = 0 the refinement is the identity, so decoding equals plain BP+LSD.
 *
 * Shapes: n and nnz below 65535 whose u16 CSR/CSC tables fit in LDS next to the weights (up to
 * about 60k edges, e.g. the 936 x 8800 detector error model).  Small graphs keep all activations
 * in LDS (inference: one wavefront per shot).  On larger ones training keeps activations in a
 * device workspace the net allocates at its first gradient call (one slice per compute unit,
 * about 6 MB each for the detector model), and inference runs one workgroup per shot over a
 * feature workspace (about 0.7 MB per compute unit for the detector model): the net's own for
 * qlsd_net_forward, the decoder's for decoding (allocated by qlsd_decoder_set_net).  Calls that
 * use the net's own workspaces (forward, gradient, train_step) must not overlap in time.
 * All device pointers are caller-owned; calls are asynchronous on `stream` unless stated.
 */
#ifndef QLSD_NET_H
#define QLSD_NET_H

#include <stdint.h>

#include "qlsd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define QLSD_NET_PARAMS 9537

typedef struct qlsd_net_s *qlsd_net;

/* priors: host double[n] (as for qlsd_decoder_create); params: host float[QLSD_NET_PARAMS]. */
qlsd_status qlsd_net_create(qlsd_code code, const double *priors, const float *params, qlsd_net *out);
qlsd_status qlsd_net_set_params(qlsd_net net, const float *params);  /* host float[QLSD_NET_PARAMS]; synchronous */
/* Replaces the priors (host double[n], each in (0,1)) that qlsd_net_forward, _gradient and
 * _train_step feed the network, e.g. to train one net over several noise strengths; synchronous. */
qlsd_status qlsd_net_set_priors(qlsd_net net, const double *priors);
qlsd_status qlsd_net_get_params(qlsd_net net, float *params);        /* host float[QLSD_NET_PARAMS]; synchronous */

/* llr_out = L + Delta for B shots: syndromes device u8[B*m], llr device float[B*n]
 * (llr_out may alias llr). */
qlsd_status qlsd_net_forward(qlsd_net net, const uint8_t *syndromes, const float *llr, int32_t B,
                             float *llr_out, void *stream);

/* Mean loss over the B shots' faults and its gradient: grad device float[QLSD_NET_PARAMS],
 * loss device float[1] (both overwritten).  errors device u8[B*n] (true error, 0/1). */
qlsd_status qlsd_net_gradient(qlsd_net net, const uint8_t *syndromes, const float *llr, const uint8_t *errors,
                              int32_t B, float *grad, float *loss, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr on the mean loss of
 * the B shots; the parameters live on the device inside the net.  Asynchronous. */
qlsd_status qlsd_net_train_step(qlsd_net net, const uint8_t *syndromes, const float *llr, const uint8_t *errors,
                                int32_t B, float lr, void *stream);

/* Attach (or, with NULL, detach) a net to a decoder of the same code (QLSD_E_INVALID if the
 * net was built for a matrix of another shape; on large graphs it allocates the decoder's
 * feature workspace, QLSD_E_NOMEM if that fails): qlsd_decode then runs
 * BP, the refinement on the shots BP did not solve, and LSD on the refined LLRs.  The attached
 * net reads the decoder's priors (not its own), so one net may serve decoders of different
 * noise strengths.  The net must outlive the attachment. */
qlsd_status qlsd_decoder_set_net(qlsd_decoder dec, qlsd_net net);

void qlsd_net_destroy(qlsd_net net);

#ifdef __cplusplus
}
#endif
#endif /* QLSD_NET_H */
