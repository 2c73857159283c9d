/* Drives every entry point of the FP64 oracle (oracle/f2v_oracle.c) over
 * small graphs and the edge cases of the method, for a build with the host
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers_cpu.py):
 * any out-of-bounds access, leak, overflow or misaligned load aborts the run.
 * Prints "ok" at the end. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t or_uniform_index(uint32_t x0, uint32_t x1, int64_t n);
int64_t or_perm_at(int64_t n, uint64_t seed, uint32_t epoch, int64_t p);
int64_t or_pos_at(int64_t n, uint64_t seed, uint32_t epoch, int64_t v);
void or_partition(int64_t n, uint64_t seed, uint32_t epoch, int mode, int32_t *perm);
void or_negatives(int64_t n, int64_t nbatches, int32_t s, uint64_t seed, uint32_t epoch, int32_t *S);
void or_eval_negatives(int64_t n, int32_t s, uint64_t seed, int32_t *W);
int32_t or_walk(const int64_t *rowptr, const int32_t *colidx, uint64_t seed, uint32_t epoch, int64_t u,
                int32_t k, int32_t *list, int32_t *raw, int32_t *nraw);
void or_loss(int64_t n, int32_t d, const int64_t *rowptr, const int32_t *colidx, const double *Z, int32_t s,
             const int32_t *W, int force, double eps, int emul, int nthreads, double out[3]);
int or_epoch(int64_t n, int32_t d, const int64_t *rowptr, const int32_t *colidx, double *Z, int32_t b, int32_t s,
             int force, double eps, double lr, uint64_t seed, uint32_t epoch, int perm_mode,
             const int32_t *S_inject, int emul, int nthreads, int64_t *pairs, int64_t k_begin, int64_t k_end,
             int32_t walk_k);
double or_learning_rate(double lr0, int schedule, int32_t epoch, int32_t total_epochs);
void or_set_num_threads(int n);

typedef struct {
  int64_t n, nnz;
  int64_t *rowptr;
  int32_t *colidx;
} Graph;

static uint64_t lcg_state = 12345;
static uint32_t lcg(void) {
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(lcg_state >> 33);
}

/* CSR from an edge list (both directions), rows in insertion order. */
static Graph from_edges(int64_t n, int64_t m, const int64_t *a, const int64_t *b) {
  Graph g;
  g.n = n;
  g.nnz = 2 * m;
  g.rowptr = calloc((size_t)n + 1, sizeof(int64_t));
  g.colidx = malloc(sizeof(int32_t) * (size_t)(g.nnz > 0 ? g.nnz : 1));
  for (int64_t i = 0; i < m; ++i) {
    g.rowptr[a[i] + 1]++;
    g.rowptr[b[i] + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) g.rowptr[v + 1] += g.rowptr[v];
  int64_t *fill = malloc(sizeof(int64_t) * (size_t)n);
  memcpy(fill, g.rowptr, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < m; ++i) {
    g.colidx[fill[a[i]]++] = (int32_t)b[i];
    g.colidx[fill[b[i]]++] = (int32_t)a[i];
  }
  free(fill);
  return g;
}

static Graph random_graph(int64_t n, int64_t m, int isolate_last) {
  int64_t *a = malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1)), *b = malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  const int64_t span = isolate_last ? n - 1 : n;
  for (int64_t i = 0; i < m; ++i) {
    a[i] = lcg() % span;
    b[i] = lcg() % span; /* self-loops and duplicates allowed */
  }
  Graph g = from_edges(n, m, a, b);
  free(a);
  free(b);
  return g;
}

static Graph star(int64_t n) {
  int64_t *a = malloc(sizeof(int64_t) * (size_t)n), *b = malloc(sizeof(int64_t) * (size_t)n);
  for (int64_t i = 1; i < n; ++i) {
    a[i - 1] = 0;
    b[i - 1] = i;
  }
  Graph g = from_edges(n, n - 1, a, b);
  free(a);
  free(b);
  return g;
}

static void release(Graph *g) {
  free(g->rowptr);
  free(g->colidx);
}

static void run_case(const Graph *g, int32_t d, int32_t b, int32_t s, int force, double eps, int emul,
                     int32_t walk_k, int perm_mode, int threads) {
  const int64_t n = g->n;
  double *Z = malloc(sizeof(double) * (size_t)n * d);
  for (int64_t i = 0; i < n * d; ++i) Z[i] = ((double)(lcg() % 2000) - 1000.0) / 2000.0;
  int64_t pairs = 0;
  for (uint32_t e = 0; e < 2; ++e) {
    int rc = or_epoch(n, d, g->rowptr, g->colidx, Z, b, s, force, eps, 0.02, 7, e, perm_mode, NULL, emul,
                      threads, &pairs, 0, -1, walk_k);
    if (rc != 0) {
      printf("or_epoch failed: %d\n", rc);
      exit(1);
    }
  }
  /* a slice of batches, and injected negatives */
  const int64_t nb = (n + b - 1) / b;
  int32_t *S = malloc(sizeof(int32_t) * (size_t)(nb * (s > 0 ? s : 1)));
  for (int64_t i = 0; i < nb * s; ++i) S[i] = (int32_t)(lcg() % n);
  if (or_epoch(n, d, g->rowptr, g->colidx, Z, b, s, force, eps, 0.02, 7, 2, perm_mode, S, emul, threads, &pairs,
               nb / 2, nb, walk_k) != 0)
    exit(1);
  free(S);
  int32_t *W = malloc(sizeof(int32_t) * (size_t)(n * (s > 0 ? s : 1)));
  or_eval_negatives(n, s, 3, W);
  double out[3];
  or_loss(n, d, g->rowptr, g->colidx, Z, s, W, force, eps, emul, threads, out);
  free(W);
  free(Z);
}

int main(void) {
  or_set_num_threads(4);
  /* random streams */
  for (int64_t n = 1; n <= 70000; n = n * 3 + 1) {
    int32_t *perm = malloc(sizeof(int32_t) * (size_t)n);
    or_partition(n, 5, 3, 0, perm);
    or_partition(n, 5, 3, 1, perm);
    (void)or_perm_at(n, 5, 3, n - 1);
    (void)or_pos_at(n, 5, 3, 0);
    free(perm);
    const int64_t nb = (n + 383) / 384;
    int32_t *S = malloc(sizeof(int32_t) * (size_t)(nb * 10));
    or_negatives(n, nb, 10, 9, 1, S);
    free(S);
  }
  (void)or_uniform_index(0xffffffffu, 0xffffffffu, 1);
  (void)or_learning_rate(0.02, 1, 9, 10);

  Graph gs[4];
  gs[0] = random_graph(300, 1500, 1); /* with an isolated vertex, self-loops, duplicates */
  gs[1] = star(200);
  gs[2] = random_graph(1, 0, 0);      /* n = 1, no edges */
  gs[3] = random_graph(50, 20, 0);    /* sparse: dead ends for the walks */
  for (int gi = 0; gi < 4; ++gi) {
    const Graph *g = &gs[gi];
    for (int force = 0; force <= 4; ++force) {
      run_case(g, 7, 32, 5, force, 1e-3, 0, 0, 0, 1);
      run_case(g, 2, 1, 0, force, 0.0, 0, 0, 1, 4);
    }
    run_case(g, 16, 1000, 3, 1, 1e-3, 1, 0, 0, 4); /* b > n, bf16 emulation */
    for (int32_t k = 1; k <= 64; k *= 4) run_case(g, 4, 17, 2, 0, 1e-3, 0, k, 0, 4);
    int32_t list[64], raw[256], nraw = 0;
    for (int64_t u = 0; u < g->n; ++u) (void)or_walk(g->rowptr, g->colidx, 11, 2, u, 64, list, raw, &nraw);
  }
  for (int gi = 0; gi < 4; ++gi) release(&gs[gi]);
  printf("ok\n");
  return 0;
}
