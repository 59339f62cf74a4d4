/*
 * exohip serving engine: continuous batching of emission-spectrum requests
 * on one GPU.  C ABI; builds on include/exohip.h.
 *
 * The workload is the one the paper's sampler generates (Sec. 5.2): a stream
 * of spectrum evaluations at nearby parameters, against line lists that stay
 * resident in GPU memory between evaluations (Sec. 2.6 keeps them on the
 * device across calls for the same reason).
 *
 * Model of operation:
 *   - Requests are queued in arrival order (exo_server_submit copies every
 *     host array it needs).
 *   - A dispatcher thread admits the preferred request as soon as a stream
 *     slot is free AND a contiguous region of the device memory budget large
 *     enough for the request's workspace is free (first fit).  The preferred
 *     request is the head of the queue (EXO_SERVE_FIFO, the default), or
 *     with EXO_SERVE_SHORTEST_FIRST the one with the fewest line x grid
 *     point x layer evaluations among the first 64 queued, unless one of
 *     those has been passed over max_passes times (then the earliest such).
 *     While the preferred request waits for memory, other requests (among
 *     the first 64) that fit may go first, at most 8 of them per waiting
 *     request; after that it is admitted before any other.  The budget is one device
 *     allocation made at creation; nothing is allocated while serving.
 *     Admitted requests run concurrently on separate HIP streams (default
 *     priority) and overlap on the device; a finished request frees its slot
 *     and region, which admits the next.
 *   - Every request runs exactly the kernels and launch shapes it would run
 *     alone, so its result is bitwise identical alone and in the mix.
 *   - The context's line lists and grid must not be changed while a server
 *     uses them.
 */
#ifndef EXOHIP_SERVE_H
#define EXOHIP_SERVE_H

#include "exohip.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct exo_server exo_server;

typedef enum {
  EXO_SERVE_FIFO = 0,           /* arrival order                                  */
  EXO_SERVE_SHORTEST_FIRST = 1  /* fewest evaluations first, passes bounded      */
} exo_serve_policy;

typedef struct {
  int64_t submitted, admitted, completed, failed, rejected;
  int64_t queued, in_flight;
  int64_t peak_in_flight; /* most requests on the device at once          */
  int64_t bypasses;       /* admissions ahead of a head waiting for memory */
  double mem_budget_bytes, mem_in_use_bytes, mem_peak_bytes;
} exo_server_counters;

/* Create a server on ctx with `n_streams` concurrent slots (1..16) and a
 * device-memory budget of `mem_budget_bytes` for request workspaces
 * (allocated once, here).  Errors: EXO_EINVAL, EXO_ENOMEM, EXO_EDEVICE. */
int exo_server_create(exo_ctx* ctx, int n_streams, size_t mem_budget_bytes, exo_server** out);

/* Admission order (see above) for the requests admitted from now on.
 * max_passes (1..2^20, EXO_SERVE_SHORTEST_FIRST): how often a request may be
 * passed over by later arrivals before it is preferred; it bounds the extra
 * wait of a large request.  Errors: EXO_EINVAL. */
int exo_server_set_policy(exo_server* srv, int policy, int max_passes);

/* Drain all queued and running requests, then release the server. */
int exo_server_destroy(exo_server* srv);

/* Queue one spectrum evaluation (as exo_emission_flux).  atm/resp and their
 * host arrays are copied; flux_dev (device, caller-owned, [out_len] float for
 * EXO_FP32_KAHAN or double for EXO_FP64) must stay valid until the request
 * has been waited for.  *ticket identifies the request.
 * arrival_s: the request's arrival time in seconds on CLOCK_MONOTONIC (the
 * clock of Python's time.monotonic()); latency and queue time are measured
 * from it.  arrival_s <= 0, or a time later than the call, means the time of
 * the call.
 * Errors: validation errors of exo_emission_flux (nothing queued);
 * EXO_ENOMEM if the request's workspace can never fit the budget. */
int exo_server_submit(exo_server* srv, const exo_atmos* atm, const exo_response* resp,
                      int precision, void* flux_dev, double arrival_s, int64_t* ticket);

/* Block until request `ticket` has finished (timeout_s < 0: no limit).
 * Returns the request's own status (EXO_OK or its error) or EXO_EINVAL for
 * an unknown ticket / timeout.  Optional outputs, in seconds since the
 * request's arrival: latency (until the GPU finished it) and queue time
 * (until admission).
 * A ticket can be waited for once. */
int exo_server_wait(exo_server* srv, int64_t ticket, double timeout_s, double* latency_s,
                    double* queue_s);

int exo_server_stats(exo_server* srv, exo_server_counters* out);

/* Workspace bytes one evaluation of (atm, resp, precision) reserves: the
 * region the server must find for it.  0 if the arguments are invalid. */
size_t exo_workspace_bytes(exo_ctx* ctx, const exo_atmos* atm, const exo_response* resp,
                           int precision);

#ifdef __cplusplus
}
#endif
#endif /* EXOHIP_SERVE_H */
