/*
 * qlsd.h -- C ABI of the MI355X BP + localized-statistics decoder (libqlsd.so).
 *
 * Problem (Hillmann et al., arXiv:2406.18655, Sec. 2.1): given a detector check
 * matrix H in F_2^{m x n}, per-fault priors p_j and a batch of syndromes s, return
 * corrections e_hat with H e_hat = s that are as likely (low weight) as the method
 * finds.  The method: min-sum belief propagation (Sec. 4.3, parallel schedule,
 * scaling 0.625), and, for shots where BP does not satisfy the syndrome, LSD on
 * BP's posterior LLRs (Sec. 4.1 / Alg. 1 with the synchronous rounds of
 * Appendix B / Alg. 2; on-the-fly elimination of Sec. 4.2), optionally followed
 * by the order-mu local reprocessing of Appendix D.
 *
 * Conventions for every entry point:
 *   - Every function returns a qlsd_status (0 = success, < 0 = error) and never
 *     throws; qlsd_last_error() gives a thread-local message for the last error.
 *   - "host" pointers are read during the call only and copied.  "device"
 *     pointers are caller-owned HIP device memory that must stay valid until the
 *     work on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Decode
 *     calls are asynchronous: argument errors are returned synchronously, device
 *     failures surface from qlsd_sync().
 *   - Decode calls never allocate: a decoder's device workspace is sized once for
 *     max_batch shots in qlsd_decoder_create().
 *   - A decoder handle is not re-entrant: calls that overlap on one decoder race
 *     on its workspace.  Distinct decoders may run concurrently on distinct streams.
 *   - Layouts are row-major, one byte per bit: syndromes B x m (values 0/1),
 *     corrections B x n (0/1), LLRs B x n float32.
 */
#ifndef QLSD_H
#define QLSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QLSD_OK = 0,
    QLSD_E_INVALID = -1,     /* bad argument, shape or matrix (e.g. a BP row of weight < 2) */
    QLSD_E_PRIOR = -2,       /* a prior outside (0, 1) */
    QLSD_E_NOMEM = -3,       /* device or host allocation failed */
    QLSD_E_DEVICE = -4,      /* a HIP call or kernel failed */
    QLSD_E_BATCH = -5,       /* B < 0 or B > max_batch */
    QLSD_E_UNSUPPORTED = -6  /* size beyond what the kernels support */
} qlsd_status;

typedef struct qlsd_code_s *qlsd_code;       /* immutable H on the device; library-owned */
typedef struct qlsd_decoder_s *qlsd_decoder; /* params, priors and workspace; library-owned */

/* Parameters (Sec. 4.3 and Appendix D). */
typedef struct {
    int32_t max_iter;   /* BP iterations, >= 1 (30 in the paper; 50/100 for larger graphs) */
    float ms_scaling;   /* min-sum scaling factor alpha (0.625 in the paper) */
    int32_t lsd_order;  /* mu: extra growth steps per cluster after LSD-0 (0 = LSD-0); with OSD-E
                           also the local search order, so at most 12; with OSD-CS at most 4096 */
    int32_t osd_method; /* local reprocessing of LSD-mu: 0 = exhaustive (OSD-E) over the first
                           min(mu, |T|) dependent columns of each cluster; 1 = combination sweep
                           (OSD-CS): every single dependent column, then pairs among the first
                           min(osd_order, |T|) (Appendix D's bivariate bicycle study) */
    uint32_t flags;     /* QLSD_FLAG_* */
    int32_t osd_order;  /* OSD-CS order w in [1, 12] (osd_method 1 only) */
} qlsd_params;

#define QLSD_FLAG_NO_EARLY_EXIT 1u /* run all max_iter BP iterations for every shot */
#define QLSD_FLAG_STAGE_TIMING 2u  /* record HIP events around each kernel of qlsd_decode */
#define QLSD_FLAG_SEPARATE_LSD 4u  /* qlsd_decode: BP and LSD as two kernels, never overlapped */
#define QLSD_FLAG_OSD0_POST 8u     /* qlsd_decode: global OSD-0 (qlsd_osd0) instead of LSD after
                                      BP, the comparator of Sec. 2.2; needs n <= 4096, m <= 1024.
                                      With osd_method 1: global OSD-CS of order osd_order
                                      (qlsd_osd_cs) instead, needs m <= 256 */

/* Per-shot status bits (qlsd_shot_info.status). */
#define QLSD_ST_BP_CONVERGED 1u /* BP's hard decision satisfies s; no LSD was needed   */
#define QLSD_ST_LSD_RUN 2u      /* LSD produced the correction                          */
#define QLSD_ST_UNSAT 4u        /* some cluster could not be made valid (s not in image) */
#define QLSD_ST_BAD_LLR 8u      /* NaN soft information; correction left at zero        */
#define QLSD_ST_OVERFLOW 16u    /* clusters outgrew even the 1024-row overflow kernel (more
                                   than 1024 clustered detectors, or more than 4096 dependent
                                   columns with LSD-mu); correction zero */

typedef struct {
    uint8_t status;           /* QLSD_ST_* bits */
    uint8_t reserved;
    int16_t bp_iters;         /* BP iterations run */
    int16_t n_clusters;       /* LSD: clusters at termination */
    int16_t rounds;           /* LSD: growth rounds */
    int32_t max_cluster_cols; /* LSD: largest cluster, in columns */
} qlsd_shot_info;             /* 12 bytes */

/* Cluster statistics of one shot (Appendix A): nu clusters, the largest of kappa faults, and the
 * size-weighted mean cluster size kappa_alpha = sumsq_cols / total_cols (the expected size of
 * the cluster a random member fault belongs to).  16 bytes. */
typedef struct {
    int32_t n_clusters; /* nu */
    int32_t max_cols;   /* kappa */
    int32_t total_cols; /* faults in all clusters */
    int32_t sumsq_cols; /* sum over clusters of the squared fault count */
} qlsd_cluster_stats;

/* H as CSR (host): row_ptr[m+1], col_idx[nnz] with columns sorted and unique per row.
 * 1 <= m, n; nnz = row_ptr[m].  Copies to the current HIP device. */
qlsd_status qlsd_code_create(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, qlsd_code *out);

/* priors: host double[n], each in (0, 1) (QLSD_E_PRIOR otherwise); the decoder uses
 * lambda_j = ln((1-p_j)/p_j) rounded to float32.  Allocates all device workspace for
 * up to max_batch shots.  The code must outlive the decoder. */
qlsd_status qlsd_decoder_create(qlsd_code code, const qlsd_params *params, const double *priors,
                                int32_t max_batch, qlsd_decoder *out);

/* BP then LSD (Sec. 2.3): syndromes device u8[B*m] -> corrections device u8[B*n];
 * info device qlsd_shot_info[B] or NULL.  0 <= B <= max_batch.
 * With slot BP and no refinement net (and without QLSD_FLAG_SEPARATE_LSD) BP and LSD share
 * one kernel: a workgroup whose BP shots have drained decodes, with LSD, the shots other
 * workgroups' BP left unsolved; a stand-alone LSD launch then finishes any shot not yet
 * taken.  Outputs are identical either way (every shot's LSD is the same function of its
 * syndrome and BP posterior).  Shots whose clusters outgrow the LSD kernel's register basis
 * (64 W local rows, W = 1, 2 or 4 chosen from m; 4 with LSD-mu; see
 * qlsd_decoder_set_lsd_capacity) are decoded again by an overflow kernel with 512 local rows
 * (basis in LDS) and, beyond that, one with 1024 (basis in device memory): same results, slower
 * per shot. */
qlsd_status qlsd_decode(qlsd_decoder dec, const uint8_t *syndromes, int32_t B, uint8_t *corrections,
                        qlsd_shot_info *info, void *stream);

/* qlsd_decode without the decoder's own device workspace, for callers that cannot allocate
 * (work under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * per-call scratch (counters, shot lists, the BP-to-LSD posterior rows, the overflow lists and
 * the 1024-row LSD bases) is carved from one static device array of the library, 48 MiB per GPU,
 * held until the process ends.  Same arguments, kernels and outputs as qlsd_decode; no
 * allocation, memset or host synchronisation.  QLSD_E_BATCH if B's scratch (at most about
 * B * (4n + 13) bytes, plus 2 MiB of bases when m > 512, or with QLSD_FLAG_OSD0_POST when
 * m > 256) exceeds 48 MiB; QLSD_E_UNSUPPORTED for a decoder whose
 * attached refinement net needs its own workspace (large graphs).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (any decoder, any stream) race. */
qlsd_status qlsd_decode_static(qlsd_decoder dec, const uint8_t *syndromes, int32_t B, uint8_t *corrections,
                               qlsd_shot_info *info, void *stream);

/* BP only: llr_out device float[B*n] receives the posterior LLRs L_j of the last
 * iteration run; hard_out device u8[B*n] (nullable) receives [L_j < 0]. */
qlsd_status qlsd_bp(qlsd_decoder dec, const uint8_t *syndromes, int32_t B, float *llr_out,
                    uint8_t *hard_out, qlsd_shot_info *info, void *stream);

/* LSD only (Alg. 1/2): soft information llr device float[B*n] (lower = more likely
 * in error; ties broken by the smaller fault index) -> corrections device u8[B*n]. */
qlsd_status qlsd_lsd(qlsd_decoder dec, const uint8_t *syndromes, const float *llr, int32_t B,
                     uint8_t *corrections, qlsd_shot_info *info, void *stream);

/* qlsd_lsd, and stats device qlsd_cluster_stats[B] receives the statistics of the clusters LSD
 * ended with (their columns: every fault a cluster took in, pivot or not; zeros for a shot
 * with no flipped detector, NaN input or overflow). */
qlsd_status qlsd_lsd_stats(qlsd_decoder dec, const uint8_t *syndromes, const float *llr, int32_t B,
                           uint8_t *corrections, qlsd_shot_info *info, qlsd_cluster_stats *stats, void *stream);

/* The optimal factorization of Appendix A for errors device u8[B*n]: the connected components
 * of each error's faults in the fault graph (faults adjacent iff they share a detector) ->
 * stats device qlsd_cluster_stats[B]. */
qlsd_status qlsd_error_clusters(qlsd_code code, const uint8_t *errors, int32_t B, qlsd_cluster_stats *stats,
                                void *stream);

/* Global OSD-0 only (Sec. 2.2, inversion decoding): on soft information llr device float[B*n]
 * (lower = more likely in error, ties broken by the smaller fault index) every column of H is
 * taken in ascending (llr_j, j), the greedy pivot set over all m detectors is formed, and
 * corrections device u8[B*n] receive the unique solution of H e = s on it (bit-exact with
 * reducing all n columns).  info: status LSD_RUN (plus UNSAT, all-zero correction, when s is not
 * in the image of H; BAD_LLR for NaN input), n_clusters 1, rounds and max_cluster_cols = the
 * columns reduced before s was spanned.  QLSD_E_UNSUPPORTED beyond n = 4096 or m = 1024. */
qlsd_status qlsd_osd0(qlsd_decoder dec, const uint8_t *syndromes, const float *llr, int32_t B,
                      uint8_t *corrections, qlsd_shot_info *info, void *stream);

/* Global OSD-CS of order `order` in [1, 12] (Sec. 2.2 and 2.3: the BP+OSD comparator at higher
 * order; the combination sweep of LSD-mu's local reprocessing applied to the whole matrix): the
 * key order and greedy pivot set of qlsd_osd0 over all n columns, T = the non-pivot columns in
 * ascending key; candidates in this order -- the OSD-0 solution, every single column of T set,
 * every pair among the first min(order, |T|) columns of T -- each fixing those columns of T to
 * one and solving the pivot part; the one of smallest integer weight sum_{e_j=1} omega_j
 * (omega_j = round(2^20 lambda_j) from the decoder's priors) wins, ties to the candidate met
 * first.  Arguments, layout and info as qlsd_osd0 (rounds and max_cluster_cols = n, every
 * column reduced).  QLSD_E_INVALID for an order outside [1, 12]; QLSD_E_UNSUPPORTED beyond
 * n = 4096 or m = 256. */
qlsd_status qlsd_osd_cs(qlsd_decoder dec, const uint8_t *syndromes, const float *llr, int32_t B, int32_t order,
                        uint8_t *corrections, qlsd_shot_info *info, void *stream);

/* Device time (ms) of the BP kernel and of the LSD kernel in the decoder's last
 * qlsd_decode call, from HIP events recorded on that call's stream around each kernel
 * (BP and LSD in one kernel: that kernel, then the stand-alone LSD launch after it).
 * Needs QLSD_FLAG_STAGE_TIMING in the decoder's params (QLSD_E_INVALID otherwise);
 * waits for those events.  Either output pointer (host float) may be NULL. */
qlsd_status qlsd_decoder_stage_ms(qlsd_decoder dec, float *bp_ms, float *lsd_ms);

/* Switches the stage events of later qlsd_decode calls on (enable != 0) or off, so that a caller
 * can time a sample of its calls without recording three events on every one (each costs a few
 * microseconds of device time).  A decoder created with QLSD_FLAG_STAGE_TIMING starts with them
 * on; QLSD_E_INVALID for one created without it.  qlsd_decoder_stage_ms then reports the last
 * call made with them on.  Not synchronised with calls in flight on other host threads. */
qlsd_status qlsd_decoder_set_stage_timing(qlsd_decoder dec, int32_t enable);

/* Autotuner: times candidate launch shapes on a sample batch (syndromes device u8[B*m],
 * B <= max_batch, typically one full batch of the workload) and keeps the fastest -- for BP
 * with shot slots, the slots per workgroup and workgroups per compute unit (timed on the whole
 * qlsd_decode when no refinement net is attached, since the shape decides whether BP and LSD
 * can share one kernel); for LSD, the number of workgroups, then the LSD capacity tier (as
 * qlsd_decoder_set_lsd_capacity, every tier up to the decoder's default, timed on the whole
 * decode; a smaller tier is kept only when it is at least 10 % faster on the sample, since other
 * batches may hold more shots that outgrow it), and at 256 rows the LSD schedule (as
 * qlsd_decoder_set_lsd_schedule; the batched one kept when 2 % faster).  Outputs never depend on these shapes.  Synchronous on `stream`;
 * allocates and frees scratch output buffers; must not overlap other calls on this decoder.
 * `report` (host char[report_len], nullable) receives one line per candidate and the choice. */
qlsd_status qlsd_decoder_tune(qlsd_decoder dec, const uint8_t *syndromes, int32_t B, int32_t reps,
                              void *stream, char *report, int32_t report_len);

/* LSD capacity tier, a schedule for uneven cluster sizes (Sec. 4.2 grows clusters of unbounded
 * size; most shots need few local rows, a few need many).  The LSD kernel holds a shot's
 * Gauss-Jordan basis in registers with room for local_rows (64, 128 or 256) clustered checks per
 * wavefront; a shot whose clusters outgrow it is handed whole to the overflow kernels (512 local
 * rows with the basis in LDS, then 1024 in device memory).  Smaller tiers run more wavefronts per compute unit and, at 64
 * or 128, let BP and LSD share one kernel; outputs never depend on the tier.  The decoder's
 * default is the smallest tier that holds every check of the code (256 when m > 128); LSD-mu
 * decoders accept 256 only (QLSD_E_UNSUPPORTED otherwise).  May allocate the overflow lists and
 * the 1024-row kernel's workspace (device memory, freed with the decoder); QLSD_E_UNSUPPORTED when
 * no overflow kernel fits the code or an allocation fails, leaving the decoder unchanged.  Host-side; must not
 * overlap other calls on this decoder. */
qlsd_status qlsd_decoder_set_lsd_capacity(qlsd_decoder dec, int32_t local_rows);

/* LSD schedule of the 256-row kernel (Sec. 4.1 and Appendix B grow every invalid cluster in a
 * round; the paper parallelises over clusters).  QLSD_LSD_PER_COLUMN (the default) reduces the
 * round's new columns one at a time in key order; QLSD_LSD_CLUSTER_BATCHED groups them so that a
 * batch holds one column per cluster and reduces a batch in one pass over the shot's local rows
 * (clusters own disjoint rows), in rounds with 4 to 64 selections.  Outputs never depend on the
 * schedule.  QLSD_E_UNSUPPORTED for the batched schedule when the capacity is below 256 local
 * rows.  Host-side; must not overlap other calls on this decoder.  qlsd_decoder_tune times both. */
#define QLSD_LSD_PER_COLUMN 0
#define QLSD_LSD_CLUSTER_BATCHED 1
qlsd_status qlsd_decoder_set_lsd_schedule(qlsd_decoder dec, int32_t schedule);

/* Waits for the decoder's last work and reports a device failure, if any. */
qlsd_status qlsd_sync(qlsd_decoder dec);

/* Thread-local text of the last error ("" if none).  Never NULL. */
const char *qlsd_last_error(void);

void qlsd_decoder_destroy(qlsd_decoder dec);
void qlsd_code_destroy(qlsd_code code);

#ifdef __cplusplus
}
#endif
#endif /* QLSD_H */
