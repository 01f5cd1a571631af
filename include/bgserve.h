/*
 * bgserve -- a request loop over the batched GEMM on one MI355X.
 *
 * The paper's application keeps many independent Monte Carlo procedures busy
 * on one GPU at once, each issuing its own sequence of products (Section III,
 * the tasked approach); its gain over lock-step batching comes from letting
 * independent sequences interleave.  This loop serves such sequences from one
 * process: clients own device-resident states, requests of different clients
 * are batched together at every step (continuous batching), and requests of
 * one client run in arrival order.
 *
 * Model.  Client c has a fixed size n_c and a state S_c (n_c x n_c,
 * column-major, ld = n_c, device memory owned by the server), the identity
 * at creation and after bs_reset.  A request (c, L) applies L factors: for
 * each, the server generates F = factor(seed, c, j) on the device, where j
 * counts the products client c has received so far, and sets S_c <- F * S_c
 * (binary64, alpha 1, beta 0, through ping-pong buffers).  Element e of the
 * column-major F is word (e mod 4) of Philox4x64-10 (Salmon et al., SC'11) at
 * counter (e div 4, j, 0, 0) and key (seed, c), mapped to
 * (2 ((w >> 11) 2^-53) - 1) * sqrt(3 / n_c) (the scale keeps the state's norm
 * of order one along long chains).
 *
 * Scheduling.  The server advances in ticks.  At each tick it admits the
 * requests whose arrival time has passed into per-client queues, starts the
 * oldest queued request of every idle client, and performs one product for
 * every client with an active request: one launch generating all of the
 * tick's factors, then one bg_dgemm_batched launch per distinct size.  A
 * request finishes at the end of the tick of its L-th product.  Results do
 * not depend on timing: each client's state is the product of its own factors
 * in order, computed with the library's fixed per-size reduction order.
 *
 * Memory.  bs_create allocates, on the handle's device, three n_c x n_c
 * buffers per client (two states, one factor) and small pointer / job arrays;
 * it refuses (BG_STATUS_ALLOC_FAILED) when their total exceeds the given HBM
 * budget.  Nothing is allocated while serving.
 *
 * Threads.  A server is driven by one host thread at a time.
 */
#ifndef BGSERVE_H
#define BGSERVE_H

#include "bgemm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bs_server* bs_server_t;

/* Creates a server for num_clients clients of sizes sizes[c] (host array,
 * each in 1..4096) on the bgemm handle h (its device and stream).  budget:
 * HBM bytes the server may hold, 0 for no limit.  Errors: INVALID_VALUE for
 * bad arguments, ALLOC_FAILED for a budget or device allocation failure. */
bg_status_t bs_create(bg_handle_t h, int num_clients, const int* sizes, unsigned long long seed,
                      unsigned long long budget, bs_server_t* out);
bg_status_t bs_destroy(bs_server_t s);

/* Device bytes the server of these sizes holds (the budget test). */
unsigned long long bs_bytes_needed(int num_clients, const int* sizes);

/* States back to the identity, product counters to zero (synchronous). */
bg_status_t bs_reset(bs_server_t s);

/* Runs an open-loop schedule to completion on the calling thread.  Request r
 * (host arrays of n_requests entries, arrival times ascending) arrives at
 * arrival_s[r] seconds after the call starts, for client client[r] with
 * chain length length[r] (>= 1).  On return out_start[r] / out_finish[r]
 * hold the seconds (from the call's start) at which its first product was
 * launched and at which its last product had completed; out_ticks (may be
 * NULL) receives the number of ticks run.  INVALID_VALUE for unsorted
 * arrivals, a bad client or length; DEVICE_ERROR for a failed HIP call. */
bg_status_t bs_run_schedule(bs_server_t s, int n_requests, const double* arrival_s,
                            const int* client, const int* length, double* out_start,
                            double* out_finish, long long* out_ticks);

/* Copies client c's state (n_c * n_c doubles, column-major) to host memory
 * (synchronous), and its product count to *products (may be NULL). */
bg_status_t bs_state(bs_server_t s, int c, double* host_out, long long* products);

/* Generates factor j of client c of size n into device memory out (n * n
 * doubles, column-major) on stream (a hipStream_t, NULL = default),
 * asynchronously: the server's generator on its own, for tests. */
bg_status_t bs_fill_factor(unsigned long long seed, int c, long long j, int n, double* out,
                           void* stream);

/* Annealing sweeps in lock step: every client receives `chain` products
 * per sweep (same factors and states as requests of that length would
 * give), `sweeps` times.  With use_graph != 0 one sweep (a factor launch and
 * one batched launch per size per product, then an update of the product
 * counters on the device) is captured once as a HIP graph -- two when chain
 * is odd, one per ping-pong parity -- and replayed on the handle's stream
 * (the capture itself runs on a private stream, since the null stream cannot
 * be captured); otherwise the same launches are issued one by one.  The results are identical either way.
 * out_seconds (may be NULL) receives the device time of the sweeps.  The
 * call allocates and frees its own small arrays and graphs (outside the
 * timed part); it is synchronous. */
bg_status_t bs_run_sweeps(bs_server_t s, int sweeps, int chain, int use_graph,
                          double* out_seconds);

/* Limits the number of requests active at once (0, the default: no limit,
 * every client with queued work is served at every tick).  With a limit,
 * the oldest startable requests start first; 1 serves one request at a
 * time in arrival order (no batching across clients, the baseline that
 * continuous batching is measured against). */
bg_status_t bs_set_max_active(bs_server_t s, int max_active);

/* Host-only replay of the scheduler on a virtual clock where every tick
 * lasts tick_s seconds, with the given max_active: fills out_start /
 * out_finish as bs_run_schedule would (tick start and end times), and
 * out_ticks.  Touches no device. */
bg_status_t bs_simulate(int num_clients, int n_requests, const double* arrival_s,
                        const int* client, const int* length, double tick_s, int max_active,
                        double* out_start, double* out_finish, long long* out_ticks);

#ifdef __cplusplus
}
#endif
#endif /* BGSERVE_H */
