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
 * requests whose arrival time has passed into per-client queues, starts
 * queued requests of idle clients (oldest first, as the policy, the active
 * limit and the factor memory allow), and performs one product for every
 * client with an active request: one launch generating all of the tick's
 * factors, then one bg_dgemm_batched launch per distinct size (or one
 * variable-size launch, bs_set_tick_launch).  A request
 * finishes at the end of the tick of its L-th product.  Two policies:
 *   BS_POLICY_CONTINUOUS  (default) a request starts as soon as its client is
 *                         idle and memory allows: requests that arrive while
 *                         others run join the next tick (continuous
 *                         batching, the paper's tasked approach);
 *   BS_POLICY_LOCKSTEP    requests start only when no request is active, so
 *                         a round of requests runs in lock step until its
 *                         longest chain ends before the next round forms (the
 *                         paper's batched approach, Section III).
 * Results do not depend on timing or policy: each client's state is the
 * product of its own factors in order, computed with the library's fixed
 * per-size reduction order.
 *
 * Memory.  bs_create allocates, on the handle's device, two n_c x n_c state
 * buffers per client (resident for the server's life), small pointer / job
 * arrays, and one factor pool.  A request holds an n_c x n_c factor of the
 * pool (256-byte aligned) from its start until its last product has
 * completed; a request that does not fit waits in its queue until running
 * requests release memory (the oldest waiting request is never overtaken).
 * With a budget, the pool is the budget minus the resident part, capped at
 * every client's factor at once; bs_create refuses (BG_STATUS_ALLOC_FAILED)
 * a budget that cannot hold the resident part plus the largest factor.  A
 * pool that holds every client's factor gives each client a fixed slot (no
 * request ever waits for memory); a smaller one is handed out first-fit, so
 * fragmentation can hold a request back beyond what the free total suggests.
 * Nothing is allocated while serving.
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

/* Device bytes a server of these sizes holds with no budget: states, arrays
 * and a factor pool holding every client's factor at once. */
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
 * timed part); it is synchronous.  Every client holds a factor of the pool
 * during the sweeps: ALLOC_FAILED when the pool cannot hold them all. */
bg_status_t bs_run_sweeps(bs_server_t s, int sweeps, int chain, int use_graph,
                          double* out_seconds);

#define BS_POLICY_CONTINUOUS 0
#define BS_POLICY_LOCKSTEP 1
/* Selects the start policy of later bs_run_schedule calls (see Scheduling). */
bg_status_t bs_set_policy(bs_server_t s, int policy);

/* Factor-pool figures: its size, the most of it in use at once since the
 * last bs_run_schedule or bs_run_sweeps began, and the number of ticks of
 * the last bs_run_schedule at which the oldest startable request waited for
 * memory.  Any pointer may be NULL. */
bg_status_t bs_memory_stats(bs_server_t s, unsigned long long* pool_bytes,
                            unsigned long long* peak_bytes, long long* waits);

#define BS_TICK_PER_SIZE 0
#define BS_TICK_VBATCHED 1
/* How a tick's products are launched: BS_TICK_PER_SIZE (default), one
 * bg_dgemm_batched per distinct client size; BS_TICK_VBATCHED, one
 * bg_dgemm_vbatched over every product of the tick (sizes uploaded with the
 * pointers, planned on the device; it uses the handle's workspace).  Results
 * are bit-identical either way. */
bg_status_t bs_set_tick_launch(bs_server_t s, int mode);

/* Limits the number of requests active at once (0, the default: no limit,
 * every client with queued work is served at every tick).  With a limit,
 * the oldest startable requests start first; 1 serves one request at a
 * time in arrival order (no batching across clients, the baseline that
 * continuous batching is measured against). */
bg_status_t bs_set_max_active(bs_server_t s, int max_active);

/* Host-only replay of the scheduler on a virtual clock where every tick
 * lasts tick_s seconds, with the given policy and max_active and, when
 * pool_bytes > 0, a factor pool of that many bytes for clients of the given
 * sizes (host array; may be NULL when pool_bytes == 0): fills out_start /
 * out_finish as bs_run_schedule would (tick start and end times), out_ticks
 * and out_mem_waits (either may be NULL).  Touches no device.
 * ALLOC_FAILED when one client's factor exceeds the pool. */
bg_status_t bs_simulate(int num_clients, const int* sizes, unsigned long long pool_bytes,
                        int policy, int n_requests, const double* arrival_s,
                        const int* client, const int* length, double tick_s, int max_active,
                        double* out_start, double* out_finish, long long* out_ticks,
                        long long* out_mem_waits);

#ifdef __cplusplus
}
#endif
#endif /* BGSERVE_H */
