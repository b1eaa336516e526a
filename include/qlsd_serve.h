/*
 * qlsd_serve.h -- continuous-batching decode service over several codes (part of libqlsd.so).
 *
 * A server owns, per registered code, "lanes": each lane is a decoder (qlsd_decoder with
 * max_batch = batch_shots), its own HIP stream, pinned host staging and device buffers for one
 * batch.  Lanes are the unit of admission by device memory, decided while the server runs: a
 * code gets one lane at registration (else registration fails with QLSD_E_NOMEM); whenever all
 * of its lanes are busy and at least half a batch of its requests has arrived, the scheduler
 * adds a lane (up to max_lanes) if the decoder workspace and batch buffers fit in what is left
 * of the server's device-memory budget; an extra lane that has been idle for the retire time
 * (20 ms by default) is freed, returning its memory to the budget for the other codes.  A
 * scheduler thread forms a batch for a lane as soon as the lane is free, from whatever requests
 * of that code have arrived (FIFO, up to batch_shots) -- requests that arrive while other
 * batches run wait and are admitted as lanes free up; nothing is dropped.  Batches of different
 * codes (and of different lanes of one code) overlap on the device.  Every decode is the BP +
 * LSD of qlsd_decode (include/qlsd.h), so a request's correction does not depend on which other
 * requests shared its batch.  Requests are either host-staged (qlsd_server_submit_many: copied
 * through pinned memory both ways) or device-resident (qlsd_server_submit_many_device: syndromes
 * and corrections stay in device memory; a batch whose requests sit in consecutive rows is
 * decoded in place, otherwise gathered with device-to-device copies).
 *
 * Arrival times make open-loop load tests possible without a host thread per request: a
 * submitted request becomes visible to the scheduler only once the server clock (microseconds
 * since qlsd_server_start) reaches its arrival time.  Latency = completion - arrival.
 *
 * Host buffers passed to qlsd_server_submit* are caller-owned and must stay valid until the
 * request's completion has been reported.  Functions return qlsd_status; qlsd_last_error()
 * describes failures.  A server handle may be used from one caller thread at a time (the
 * scheduler thread is internal).
 */
#ifndef QLSD_SERVE_H
#define QLSD_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "qlsd.h"
#include "qlsd_net.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qlsd_server_s *qlsd_server;

typedef struct {
    uint64_t tag;        /* caller's request id */
    int32_t code_id;     /* as returned by qlsd_server_add_code */
    uint8_t status;      /* QLSD_ST_* bits of the shot */
    uint8_t reserved[3];
    double arrival_us;   /* server clock */
    double done_us;      /* server clock when the scheduler saw the batch finish */
    int32_t batch_size;  /* shots in the batch that carried this request */
    int32_t reserved2;
} qlsd_completion;       /* 40 bytes */

/* device_budget_bytes: device memory the lanes of all codes may use (decoder workspace plus
 * one batch of buffers per lane).  Each lane has its own stream; HIP maps streams onto hardware
 * queues (GPU_MAX_HW_QUEUES per process, 4 by default), and lanes that share a queue wait behind
 * each other's batches, so a process serving more than four lanes should raise it (e.g. to 8)
 * before HIP initialises. */
qlsd_status qlsd_server_create(size_t device_budget_bytes, qlsd_server *out);

/* Registers a code with decoder parameters and priors (host, n doubles; copied).  Creates its
 * first lane now; the scheduler adds lanes up to max_lanes while the budget allows (see above).
 * Each lane decodes batches of at most batch_shots shots.  *code_id receives the code's id;
 * *lanes_out (nullable) the lanes created now (1). */
qlsd_status qlsd_server_add_code(qlsd_server s, qlsd_code code, const qlsd_params *params,
                                 const double *priors, int32_t batch_shots, int32_t max_lanes,
                                 int32_t *code_id, int32_t *lanes_out);

/* Attaches a learned LLR refinement (include/qlsd_net.h, built for the same code) to every lane
 * of code_id (and to the lanes it gets later), or detaches it with net = NULL; only before
 * qlsd_server_start.  The net is shared
 * read-only by the lanes and must outlive the server.  On large graphs each lane's decoder gets a
 * feature workspace, charged to the device budget (QLSD_E_NOMEM if it does not fit). */
qlsd_status qlsd_server_set_net(qlsd_server s, int32_t code_id, qlsd_net net);

/* Queues count requests of one code: syndromes host u8[count*m], corrections_out host
 * u8[count*n] (written on completion), tags[count], arrival_us[count] (server clock; NULL =
 * all arrive immediately).  Arrival times of one code must be non-decreasing. */
qlsd_status qlsd_server_submit_many(qlsd_server s, int32_t code_id, int32_t count,
                                    const uint8_t *syndromes, uint8_t *corrections_out,
                                    const uint64_t *tags, const double *arrival_us);

/* As qlsd_server_submit_many with device-resident requests: syndromes device u8[count*m] and
 * corrections_out device u8[count*n] (caller-owned, valid until the completions are reported);
 * no host staging or PCIe copies.  A batch holds requests of one kind only. */
qlsd_status qlsd_server_submit_many_device(qlsd_server s, int32_t code_id, int32_t count,
                                           const uint8_t *syndromes, uint8_t *corrections_out,
                                           const uint64_t *tags, const double *arrival_us);

/* Lanes of a code: *now currently held, *created and *retired so far (each nullable). */
qlsd_status qlsd_server_lanes(qlsd_server s, int32_t code_id, int32_t *now, int32_t *created, int32_t *retired);

/* Idle time (microseconds) after which an extra lane is freed; only before qlsd_server_start. */
qlsd_status qlsd_server_set_retire_us(qlsd_server s, double retire_us);

/* Starts the scheduler thread; the server clock starts at 0 here. */
qlsd_status qlsd_server_start(qlsd_server s);

/* Blocks until at least `count` requests have completed in total, or timeout_s elapses
 * (QLSD_E_DEVICE then, with a message).  Device failures are reported here too. */
qlsd_status qlsd_server_wait(qlsd_server s, int64_t count, double timeout_s);

/* Moves up to max completion records (oldest first) into out; *n_out receives how many. */
qlsd_status qlsd_server_completions(qlsd_server s, qlsd_completion *out, int32_t max, int32_t *n_out);

/* Current server clock in microseconds (0 before start). */
double qlsd_server_now_us(qlsd_server s);

/* Stops the scheduler after the in-flight batches finish and frees every lane. */
void qlsd_server_destroy(qlsd_server s);

#ifdef __cplusplus
}
#endif
#endif /* QLSD_SERVE_H */
