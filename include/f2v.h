/*
 * f2v.h -- C ABI of the MI355X Force2Vec minibatch update.
 *
 * The library trains a graph embedding Z (n x d) with the negative-sampling
 * Force2Vec method: Algorithm 1 (epoch loop: random partition of the vertices
 * into ceil(n/b) minibatches; per batch one shared set S_b of s uniform
 * negative samples; gradient of every batch vertex; SGD step of Eq. 10 on the
 * batch vertices only) driving Algorithm 2 (per-vertex gradient: attractive
 * force over the CSR neighbours, Eq. 5 sigmoid or Eq. 8 Student-t, plus
 * repulsive force over S_b, Eq. 6 or Eq. 9).  The semantics are the paper's
 * synchronous minibatch SGD (Section 3.2): every gradient of batch k reads the
 * embedding as left by batches 0..k-1, so the result does not depend on how
 * the device schedules the work.
 *
 * Conventions
 *  - Device pointers are HIP device memory owned by the caller, alive until
 *    f2v_destroy.  The library allocates no device memory: all state lives in
 *    the caller's workspace (size from f2v_workspace_size).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *    asynchronous on that stream except f2v_init, f2v_loss, f2v_check and the
 *    host-only queries.
 *  - Every call returns f2v_status; no exception crosses the ABI.  On error
 *    f2v_last_error(ctx) (or f2v_last_error(NULL) for calls without a context)
 *    holds a message.
 *  - Argument validation runs on the host before any HIP call.
 *  - One host thread per context; distinct contexts are independent.
 *
 * Random streams (identical on every run and device; the epoch index is an
 * argument, so a run resumed at epoch e equals an uninterrupted one):
 *  - Philox4x32-10 (Salmon et al., SC'11) keyed by `seed`.
 *  - Partition of epoch e: position p -> vertex perm_e(p), a 12-round keyed
 *    Feistel permutation of [0, 2^(2h)) (round r value Philox(e, r, R, 1).x0
 *    masked to h bits) restricted to [0, n) by cycle walking; batch k holds
 *    positions [k b, min(n, (k+1) b)).  F2V_PERM_IDENTITY uses perm_e(p) = p.
 *  - Negatives of batch k in epoch e: S[k][j] = floor(w * n / 2^64) with w the
 *    64-bit word x0:x1 of Philox(e, k, j, 2), j < s (uniform, with
 *    replacement; u itself or a neighbour may be drawn).
 *  - Loss negatives of vertex u: W[u][j] from Philox(u_lo, u_hi, j, 3).
 */
#ifndef F2V_H
#define F2V_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    F2V_OK = 0,
    F2V_E_INVALID_ARG = 1, /* a parameter or pointer is out of range */
    F2V_E_BAD_GRAPH = 2,   /* CSR malformed: rowptr[0] != 0, decreasing rowptr,
                              rowptr[n] != nnz, or a column index outside [0, n) */
    F2V_E_OOM = 3,         /* workspace smaller than f2v_workspace_size */
    F2V_E_HIP = 4,         /* a HIP runtime call failed */
    F2V_E_STATE = 5,       /* call not valid in the context's state */
    F2V_E_TIMEOUT = 6,     /* a device-side dependency wait exceeded its bound;
                              the embedding is not valid after this */
    F2V_E_BUSY = 7,        /* serving: no free slot or memory for the job */
    F2V_E_UNSUPPORTED = 8  /* valid request the library does not implement */
} f2v_status;

/* Force models.  SIGMOID: Eqs. 3, 5, 6.  STUDENT_T: Eqs. 7-9 along the unit
 * vector of z_u - z_v.  The spring-electrical models of Table 2: attraction
 * of magnitude t^2 (FR, Fruchterman-Reingold), log(1 + t) (LINLOG) or t
 * (FORCEATLAS) pulling u toward a neighbour, repulsion of magnitude 1/t
 * pushing it away from a negative, t = |z_u - z_other|; the repulsion is
 * regularised as the gradient of -log(q + eps)/2, q = t^2 (0 at q + eps = 0).
 * Their loss (f2v_loss) is the potential whose gradient the forces are:
 * t^3/3, (1 + t) log(1 + t) - t or t^2/2, and -log(q + eps)/2. */
typedef enum {
    F2V_FORCE_SIGMOID = 0,
    F2V_FORCE_STUDENT_T = 1,
    F2V_FORCE_FR = 2,
    F2V_FORCE_LINLOG = 3,
    F2V_FORCE_FORCEATLAS = 4
} f2v_force;
typedef enum { F2V_FP32 = 0, F2V_BF16 = 1 } f2v_precision;
typedef enum { F2V_LR_CONST = 0, F2V_LR_LINEAR = 1 } f2v_lr_schedule;
typedef enum { F2V_PERM_RANDOM = 0, F2V_PERM_IDENTITY = 1 } f2v_perm_mode;
/* Device scheduling of one epoch; all give bit-identical results.
 * DATAFLOW: one persistent launch per epoch, sized to the update kernel's
 *   occupancy limit; batches overlap on the device and a vertex row is read
 *   only once the batch that updates it has published it; work is assigned to
 *   waves statically in batch order.  The launch first checks that its whole
 *   grid is resident at once (which the static order needs); if not, that
 *   launch hands out work as DYNAMIC does and f2v_check lowers the grid.
 * STRICT: one launch per batch, batches separated by the stream order.
 * DYNAMIC: as DATAFLOW, but running waves claim work in batch order from a
 *   counter, so the launch needs no co-residency and its grid is sized to the
 *   graph; for many concurrent jobs on one device (the server).
 * HOGWILD: the relaxed, asynchronous variant that Section 3.2 contrasts with
 *   the synchronous one: one embedding buffer updated in place, and a row is
 *   read in whatever state it is when read (no waits for earlier batches),
 *   so results depend on timing and are not reproducible; a throughput study,
 *   not the paper's method. */
typedef enum {
    F2V_SCHED_DATAFLOW = 0,
    F2V_SCHED_STRICT = 1,
    F2V_SCHED_DYNAMIC = 2,
    F2V_SCHED_HOGWILD = 3
} f2v_schedule;

typedef struct {
    int64_t n;            /* vertices, >= 1, < 2^29 - 1 */
    int64_t nnz;          /* stored CSR entries (2m for a simple undirected graph) */
    int32_t d;            /* embedding dimension: d % 4 == 0 up to 1024, d % 4 == 2
                             up to 128, odd d up to 64 (BF16: even d only) */
    int32_t batch;        /* minibatch size b >= 1 */
    int32_t s;            /* shared negatives per batch, 0..64 */
    int32_t force;        /* f2v_force */
    int32_t precision;    /* f2v_precision */
    int32_t lr_schedule;  /* f2v_lr_schedule: eta_e = lr0 or lr0 (1 - e / total_epochs) */
    float lr0;            /* initial step size eta > 0 (the paper uses 0.02) */
    float eps;            /* Student-t repulsion regulariser, 0 <= eps < 1: the
                             repulsive force is the gradient of
                             log(1+q) - log(q+eps), q = |z_u - z_w|^2; eps = 0 is
                             Eq. 9 exactly (taken as 0 at q = 0) */
    int32_t total_epochs; /* E of the linear schedule (>= 1 if linear) */
    int32_t perm_mode;    /* f2v_perm_mode */
    int32_t schedule;     /* f2v_schedule */
    int32_t chunk;        /* neighbours per work unit; rows of higher degree are
                             split into several units whose partial sums are
                             combined in a fixed order.  0 = default: 64 for
                             n >= 750000, else 32. */
    uint64_t seed;        /* key of every random stream */
    int32_t late_window;  /* split rows: the neighbours of this many batches
                             before the row's own are taken last, by the unit
                             that takes the step (0 .. 2^20); < 0 = default:
                             28 for n >= 750000, else 24.  Results do not
                             depend on it. */
    int32_t fan_in;       /* fan-in of the fixed-order tree that combines a
                             split row's partial sums, 4 .. 64; 0 = default 8 */
    int32_t walk_length;  /* 0: N(u) is u's CSR row.  k in 1 .. 64: N(u) is the
                             random-walk neighbourhood of Algorithm 3
                             (rForce2Vec), drawn afresh every epoch: the
                             distinct vertices a walk from u reaches, in the
                             order first reached (step i of epoch e from u
                             draws Philox(e, u, i, 5) and moves to the
                             neighbour at that uniform index of the current
                             row), until k are found, 4k steps are taken or
                             the walk reaches a vertex without neighbours.
                             f2v_loss still sums over the CSR rows. */
    int32_t stage_negatives; /* How a batch's s negative rows reach its units
                             (Algorithm 2, second loop).  0 (default): they
                             are the tail of every whole and late unit's list,
                             read like neighbours through the caches.  1: a
                             pass of their own before the neighbours, with the
                             rows staged once per workgroup and batch in LDS
                             and read there by the workgroup's other waves.
                             2: the same pass with every unit reading the rows
                             from memory (1 and 2 give the same bits; both
                             differ from 0 in summation order only).  1 and 2
                             need s * d <= 2048 and a schedule other than
                             dynamic; measured slower than 0 on the
                             benchmarked workloads. */
} f2v_params;

typedef struct f2v_ctx f2v_ctx;

/* Fill `p` with defaults: b = 384, s = 5, sigmoid, FP32, lr0 = 0.02 constant,
 * eps = 1e-3, random partition, dataflow schedule, chunk 0 (by size), seed 0,
 * late_window -1 and fan_in 0 (defaults), walk_length 0 (CSR rows),
 * stage_negatives 0.  n, nnz and d must still be set. */
void f2v_default_params(f2v_params *p);

/* Host only.  Step size eta_e of epoch `epoch` (Algorithm 1 fixes only the
 * initial eta): lr0, or lr0 (1 - epoch / total_epochs) under the linear
 * schedule.  F2V_E_INVALID_ARG for epoch < 0 and, under the linear schedule,
 * for epoch >= total_epochs (eta would be <= 0: no step, or ascent);
 * f2v_epoch refuses such an epoch the same way. */
f2v_status f2v_step_size(const f2v_params *p, int32_t epoch, float *eta);

/* Host only.  Bytes of device workspace the context needs (a bound from
 * n, nnz, d, b, s, precision and chunk; independent of the graph's degrees). */
f2v_status f2v_workspace_size(const f2v_params *p, size_t *bytes);

/* Create a context on the current HIP device for the problem of Section 2.1
 * (graph G(V, E) with binary symmetric adjacency A, embedding Z of n rows of
 * d) and the inputs of Algorithm 1 (b, s, the step size eta, the random
 * partition per epoch).
 *   d_rowptr : int64[n+1] CSR row offsets (device)
 *   d_colidx : int32[nnz] column indices (device); row u lists N(u)
 *   d_z      : float[n*d] row-major initial embedding (device, in/out).  FP32:
 *              the library alternates between d_z and a workspace copy;
 *              f2v_sync_embedding makes d_z current.  BF16: d_z holds the FP32
 *              master rows and is updated in place; bf16 copies feed the forces.
 *   d_ws, ws_bytes : workspace (device, >= f2v_workspace_size bytes, 256-byte aligned)
 * Validates the CSR on the device and synchronises the stream once. */
f2v_status f2v_init(const f2v_params *p, const int64_t *d_rowptr, const int32_t *d_colidx,
                    float *d_z, void *d_ws, size_t ws_bytes, void *stream, f2v_ctx **out);

/* One epoch of Algorithm 1 with epoch index `epoch` (>= 0): partition,
 * negatives, and the ceil(n/b) batch updates.  Asynchronous.  The result
 * depends only on the current embedding, the epoch index and the params. */
f2v_status f2v_epoch(f2v_ctx *ctx, int32_t epoch);

/* Loss of Eq. 2 on the current embedding, with s fixed loss negatives per
 * vertex (W above): out[0] = total, out[1] = attractive, out[2] = repulsive.
 * Per-pair terms in FP32, sums in FP64 in a fixed order.  BF16: evaluated on
 * the bf16 rows the forces read.  Synchronises the stream. */
f2v_status f2v_loss(f2v_ctx *ctx, double out[3]);

/* Make d_z hold the current embedding (FP32: a device copy if the current
 * buffer is the workspace one).  Asynchronous. */
f2v_status f2v_sync_embedding(f2v_ctx *ctx);

/* Synchronise the stream and report a device-side error raised since the
 * last check (F2V_E_TIMEOUT for an exceeded dependency wait).  A wait is
 * bounded by a count of polls (2^20, about half a second of polling), not by a
 * clock, so a wave that is suspended cannot time out.  After such a wait,
 * later epochs of the context do nothing until this check, so the failed
 * epoch's vertex words are kept: f2v_last_error then gives how many vertices
 * were never published and the earliest of them.  (In the dataflow and
 * dynamic schedules, narrow rows are their own publication: FP32 rows of
 * d <= 64 with d even or d <= 32, bf16 rows of d <= 32.  The next buffer is
 * first set to a signalling-NaN pattern, so after a failed epoch the rows it
 * never stored hold that pattern.)  If a dataflow launch since
 * the last check found its grid not co-resident, later epochs use one block
 * per CU fewer. */
f2v_status f2v_check(f2v_ctx *ctx);

/* Health record of the context (synchronises the stream): out[0] dataflow
 * launches that found their grid not co-resident and handed work out by
 * claiming instead (same results); out[1] dependency waits of the dynamic
 * schedule that polled more than 256 times (how long units wait under load);
 * out[2], out[3] reserved (0).
 * *blocks_per_cu (may be NULL): the dataflow grid's current blocks of 256
 * threads per CU. */
f2v_status f2v_health(f2v_ctx *ctx, uint32_t out[4], int32_t *blocks_per_cu);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): a whole run of the method
 * -- the checks and setup of f2v_init, epochs first_epoch .. first_epoch +
 * epochs - 1 as f2v_epoch runs them, f2v_sync_embedding and f2v_check --
 * with its workspace in a static device array of the library instead of a
 * caller's buffer.  The array holds 256 MiB (268435456 bytes) on every device
 * the library runs on, from the first call on that device until the process
 * ends; a job whose f2v_workspace_size is larger is refused with F2V_E_OOM
 * before any device work.  The call allocates no device memory and creates no
 * HIP events; it synchronises `stream` (at the CSR check and at the end).
 * d_rowptr, d_colidx, d_z as f2v_init (d_z receives the result: the FP32
 * embedding, or the FP32 master rows in the bf16 form).  Every call on a
 * device shares that device's array, which keeps the last call's contents
 * (each call initialises what it reads): calls that overlap on one device
 * race and must not be issued.  Returns the first error (F2V_E_TIMEOUT with
 * the message of f2v_check). */
f2v_status f2v_train_static(const f2v_params *p, const int64_t *d_rowptr, const int32_t *d_colidx, float *d_z,
                            int32_t first_epoch, int32_t epochs, void *stream);

/* Release the context (no device memory to free; the caller owns it). */
f2v_status f2v_destroy(f2v_ctx *ctx);

const char *f2v_status_string(f2v_status st);
const char *f2v_last_error(const f2v_ctx *ctx);

/* Device copies of the random streams an epoch uses, for checking them.
 *   f2v_partition : d_perm int32[n], perm_e(p) for every position p
 *   f2v_negatives : d_S int32[ceil(n/b) * s], S[k][j] at k*s + j
 * Asynchronous on `stream`. */
f2v_status f2v_partition(int64_t n, uint64_t seed, int32_t epoch, int32_t perm_mode,
                         int32_t *d_perm, void *stream);
f2v_status f2v_negatives(int64_t n, int32_t batch, int32_t s, uint64_t seed, int32_t epoch,
                         int32_t *d_S, void *stream);

/* Device self-test of the publication protocol that keeps the update's reads
 * exact while batches overlap (the synchronous minibatch semantics of
 * Algorithm 1 on a device whose XCDs have caches that are not coherent with
 * each other).  `pairs` pairs of single-wave workgroups, writer and reader
 * on different XCDs, run `rounds` rounds: the writer publishes a 512-byte
 * row exactly as the update kernel publishes a wide updated row (d = 128)
 * and a split row's early sum (device-scope
 * row stores, wait for their completion, device-scope flag store), the
 * reader polls the flag and reads the row as a dependent unit does, checks
 * every word, and acknowledges.  1 <= pairs <= 1024, 1 <= rounds <= 2^24.
 * d_ws: caller's device buffer, 256-byte aligned, of at least
 * 512 * pairs + 4 * (2 * pairs + 3) bytes.  out (host): [0] words read
 * stale, [1] polls that ran into the wait bound, [2] readers that completed
 * every round (a sound device gives 0, 0, pairs).  Synchronises `stream`. */
f2v_status f2v_selftest_publish(int32_t pairs, int32_t rounds, void *d_ws, size_t ws_bytes, uint32_t out[3],
                                void *stream);

/* Device copy of the random-walk neighbourhoods of epoch e (walk mode,
 * Algorithm 3; see walk_length): for every vertex u, d_len[u] <= k and its
 * walk's distinct vertices in the order first reached at d_list[u*k .. u*k +
 * d_len[u]).  d_rowptr int64[n+1] and d_colidx int32[rowptr[n]] are the CSR
 * (device), d_list int32[n*k], d_len int32[n] (device).  1 <= k <= 64.
 * Asynchronous on `stream`. */
f2v_status f2v_walks(const int64_t *d_rowptr, const int32_t *d_colidx, int64_t n, int32_t k, uint64_t seed,
                     int32_t epoch, int32_t *d_list, int32_t *d_len, void *stream);

/* A random initial embedding on the device: count floats uniform on
 * [-scale, scale) (the method starts from a random Z; a U[-0.5, 0.5) start is
 * scale 0.5).  Element i uses word i mod 4 of Philox(i div 4, 0, 0, 4) keyed by
 * seed (24 high bits).  Asynchronous on `stream`. */
f2v_status f2v_random_embedding(float *d_z, int64_t count, uint64_t seed, float scale, void *stream);

/* Device time of the most recent f2v_epoch's update kernel(s) in ms, measured
 * with HIP events on the context's stream (prologue excluded).  Synchronises. */
f2v_status f2v_last_epoch_ms(f2v_ctx *ctx, float *update_ms, float *total_ms);

/* Diagnostics.  With diagnostics on, each dataflow epoch records 8 counters
 * per wave of its update kernel (uint64): [0] cycles of the wave, [1] cycles
 * waiting for rows of earlier batches to be published, [2] cycles combining
 * split rows, [3] work groups processed, [4] polls that found a row
 * unpublished, [5] waits that had to poll, [6] cycles storing and publishing
 * rows, [7] cycles of [1] spent in units that take a split row's step.
 * f2v_wave_stats copies min(cap_waves, waves) rows of the
 * last such epoch to host memory `out` (may be NULL to query the count) and
 * synchronises the stream. */
f2v_status f2v_set_diagnostics(f2v_ctx *ctx, int32_t enable);
f2v_status f2v_wave_stats(f2v_ctx *ctx, uint64_t *out, int64_t cap_waves, int64_t *n_waves);
/* Per-vertex timeline of the last epoch run with diagnostics on, in ticks of
 * the device's constant wall clock (100 MHz on MI355X; low 32 bits): out[2u]
 * = end of the last dependency wait of the unit that finished vertex u (0 if
 * it did not wait), out[2u+1] = publication of u's new row.  `out` is host
 * memory for 2n uint32.  Synchronises. */
f2v_status f2v_vertex_trace(f2v_ctx *ctx, uint32_t *out);

/* ---------------------------------------------------------------------------
 * Serving: many embedding jobs on one device.
 *
 * A server owns `max_slots` slots, each with its own HIP stream (default
 * priority), and admits jobs while a slot is free and the sum of the admitted
 * jobs' footprints stays within `hbm_budget` bytes.  The caller allocates each
 * job's device memory (CSR, initial embedding, workspace) after checking that
 * the server can admit it, and keeps it alive until the job is reported done.
 * Jobs overlap on the device: every job runs the dynamic schedule (no
 * co-residency needed).  A job's result does not depend on the other jobs
 * running with it (bit-identical to running it alone).
 */
typedef struct f2v_server f2v_server;

/* Device bytes of one job: CSR (8(n+1) + 4 nnz), embedding (4 n d) and
 * workspace (f2v_workspace_size).  Host only. */
f2v_status f2v_footprint(const f2v_params *p, size_t *bytes);

/* Create a server (1 <= max_slots <= 256, hbm_budget > 0).  Allocates the
 * slots' streams, eight streams for the concurrent update launches of pack
 * graphs, sixteen argument-table buffers for packs (about 1 MiB each, device
 * memory plus its pinned host source) and a small pinned host array for
 * completion records. */
f2v_status f2v_server_create(size_t hbm_budget, int32_t max_slots, f2v_server **out);

/* Admit one job of `epochs` epochs (0 .. epochs-1) with params p
 * (p->schedule must be F2V_SCHED_DYNAMIC) on the caller's device buffers (as
 * f2v_init).  F2V_E_BUSY if no slot is free or the footprint does not fit the
 * remaining budget (the caller queues the job and retries).  pack == 0: the
 * run is issued at once on the slot's stream.  pack != 0: the job waits for
 * f2v_server_flush.  On success *job_id identifies the job.  Validates the
 * CSR (synchronises the slot's stream). */
f2v_status f2v_server_submit(f2v_server *s, const f2v_params *p, const int64_t *d_rowptr,
                             const int32_t *d_colidx, float *d_z, void *d_ws, size_t ws_bytes,
                             int32_t epochs, int32_t pack, uint64_t *job_id);

/* Launch the packed jobs submitted since the last flush.  They are grouped
 * into packs of jobs of similar size (n * d within a factor of 4; up to 64
 * jobs and 2048 (job, epoch) pairs per pack), and each pack is one HIP graph
 * on the slot stream of its first job that runs its jobs in lockstep epochs.
 * Per epoch the graph holds one launch of each prologue kernel for all of
 * the pack's jobs, and one multi-job update launch per kernel instance (the
 * jobs of one embedding width, precision and force family) on concurrent
 * streams.  Every job keeps its own dynamic schedule on its own workgroups,
 * so its result is the bits it gets alone.  Each job's completion record is
 * written after its own last epoch.  A job of more than 2048 epochs runs
 * alone on its slot's stream.  Waits for a running pack only when all
 * sixteen table buffers are in use. */
f2v_status f2v_server_flush(f2v_server *s);

/* Non-blocking: report up to `cap` jobs that finished (done[i], status[i] =
 * F2V_OK or F2V_E_TIMEOUT), release their slots and budget.  A finished
 * job's embedding buffer holds its result (the FP32 master in the bf16 form).
 * For a job that ended in F2V_E_TIMEOUT, f2v_server_last_error gives the
 * unpublished vertices of its failed epoch, as f2v_check does. */
f2v_status f2v_server_poll(f2v_server *s, uint64_t *done, int32_t *status, int32_t cap,
                           int32_t *n_done);

/* The health records (see f2v_health) of the jobs reported by
 * f2v_server_poll so far, summed: out[0] .. out[3]. */
f2v_status f2v_server_health(f2v_server *s, uint64_t out[4]);

/* Current occupancy (any pointer may be NULL). */
f2v_status f2v_server_query(f2v_server *s, int32_t *active, int32_t *free_slots,
                            size_t *used_bytes, size_t *budget_bytes);

/* Flush, then wait until every submitted job has finished on the device
 * (their completions are still reported by f2v_server_poll). */
f2v_status f2v_server_drain(f2v_server *s);

f2v_status f2v_server_destroy(f2v_server *s);
const char *f2v_server_last_error(const f2v_server *s);

#ifdef __cplusplus
}
#endif
#endif /* F2V_H */
