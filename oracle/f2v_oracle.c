/*
 * Force2Vec reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of one training run of
 * the paper's negative-sampling Force2Vec method (Algorithm 1 driving
 * Algorithm 2, Section 3), used to check the HIP path.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never does.  It shares no code with the HIP path.
 *
 * What it computes (each function cites the passage it follows):
 *   - per-pair forces of the sigmoid model (Eqs. 5-6) and of the Student-t
 *     model (Eqs. 8-9, times the unit vector of z_u - z_v as Section 3.2
 *     prescribes), with an optional epsilon that regularises the Student-t
 *     repulsion at zero distance;
 *   - synchronous minibatch SGD (Section 3.2, Algorithm 1): per epoch a random
 *     partition into ceil(n/b) batches, one shared set of s uniform negative
 *     samples per batch, gradients of every batch vertex taken from the state
 *     at the start of the batch (Algorithm 2), then the step of Eq. 10 applied
 *     to the batch vertices only;
 *   - the negative-sampled loss of Eq. 2 (Eqs. 3 and 7), with a fixed set of
 *     evaluation negatives per vertex so that it is a function of Z alone;
 *   - the other spring-electrical models of Table 2 (Fruchterman-Reingold,
 *     LinLog, ForceAtlas): attractive force magnitude t^2, log(1 + t) or t and
 *     repulsive magnitude 1/t along the unit vector of z_u - z_other, pulling u
 *     toward a neighbour and pushing it away from a negative; each is the
 *     gradient of a stated potential, which serves as their loss;
 *   - random-walk neighbourhoods (Algorithm 3, rForce2Vec of Section 3.3): the
 *     distinct vertices a walk from u reaches, in the order first reached,
 *     until k are found, a step bound is reached or the walk is stuck.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written from that paper's definition;
 * the partition is a keyed 12-round Feistel network on the next even power of
 * two, restricted to [0, n) by cycle walking.
 *
 * Precision: all embedding arithmetic in FP64.  The optional bf16 emulation
 * mode rounds every force input to bfloat16 (round to nearest even) while the
 * state stays FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_SIGMOID 0
#define OR_STUDENT_T 1
#define OR_FR 2          /* Fruchterman-Reingold (Table 2) */
#define OR_LINLOG 3      /* LinLog (Table 2) */
#define OR_FORCEATLAS 4  /* ForceAtlas (Table 2) */

#define TAG_PERM 1u
#define TAG_NEG 2u
#define TAG_EVAL 3u
#define TAG_WALK 5u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the SC'11 definition: ten rounds, each multiplying two
 * counter words by fixed odd constants and mixing high halves with the other
 * words and the round key; the key is bumped by Weyl constants between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_call(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                        uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* Uniform index in [0, n) from two 32-bit words: the high 64 bits of the
 * 128-bit product of the 64-bit word x0:x1 and n. */
int64_t or_uniform_index(uint32_t x0, uint32_t x1, int64_t n)
{
    unsigned __int128 w = ((unsigned __int128)(((uint64_t)x0 << 32) | x1)) * (uint64_t)n;
    return (int64_t)(w >> 64);
}

/* ------------------------------------------------------------------------ */
/* Random partition of Algorithm 1 (minibatches drawn without replacement,
 * afresh in every epoch): position -> vertex map perm_e. */

static int feistel_half_bits(int64_t n)
{
    int bits = 0;
    while (bits < 62 && ((int64_t)1 << bits) < n) ++bits;
    if (bits < 2) bits = 2;
    if (bits & 1) ++bits;
    return bits / 2;
}

static uint64_t feistel_round_fn(uint64_t seed, uint32_t epoch, uint32_t round, uint64_t r,
                                 uint64_t mask)
{
    uint32_t out[4];
    philox_call(seed, epoch, round, (uint32_t)r, TAG_PERM, out);
    return (uint64_t)out[0] & mask;
}

/* Number of Feistel rounds.  Twelve rather than the classical four: with the
 * tiny half-widths of small graphs a four-round network is visibly biased
 * (pairs of positions far from uniform), twelve rounds are not. */
#define FEISTEL_ROUNDS 12

/* One pass of the network on [0, 4^h). */
static uint64_t feistel_forward(uint64_t seed, uint32_t epoch, int h, uint64_t x)
{
    uint64_t mask = ((uint64_t)1 << h) - 1;
    uint64_t L = x >> h, R = x & mask;
    for (uint32_t r = 0; r < FEISTEL_ROUNDS; ++r) {
        uint64_t nl = R;
        uint64_t nr = L ^ feistel_round_fn(seed, epoch, r, R, mask);
        L = nl; R = nr;
    }
    return (L << h) | R;
}

static uint64_t feistel_backward(uint64_t seed, uint32_t epoch, int h, uint64_t y)
{
    uint64_t mask = ((uint64_t)1 << h) - 1;
    uint64_t L = y >> h, R = y & mask;
    for (int r = FEISTEL_ROUNDS - 1; r >= 0; --r) {
        uint64_t pl = R ^ feistel_round_fn(seed, epoch, (uint32_t)r, L, mask);
        uint64_t pr = L;
        L = pl; R = pr;
    }
    return (L << h) | R;
}

/* perm_e[p] for one position: cycle-walk the network until it lands in [0, n). */
int64_t or_perm_at(int64_t n, uint64_t seed, uint32_t epoch, int64_t p)
{
    int h = feistel_half_bits(n);
    uint64_t x = (uint64_t)p;
    do { x = feistel_forward(seed, epoch, h, x); } while (x >= (uint64_t)n);
    return (int64_t)x;
}

/* Inverse: position of vertex v. */
int64_t or_pos_at(int64_t n, uint64_t seed, uint32_t epoch, int64_t v)
{
    int h = feistel_half_bits(n);
    uint64_t x = (uint64_t)v;
    do { x = feistel_backward(seed, epoch, h, x); } while (x >= (uint64_t)n);
    return (int64_t)x;
}

/* Full partition for an epoch.  mode 0: keyed random permutation; mode 1:
 * identity (batches are consecutive vertex ranges). */
void or_partition(int64_t n, uint64_t seed, uint32_t epoch, int mode, int32_t *perm)
{
    for (int64_t p = 0; p < n; ++p)
        perm[p] = (int32_t)(mode == 1 ? p : or_perm_at(n, seed, epoch, p));
}

/* Shared negative samples of Algorithm 1 (one set of s uniform vertices per
 * batch, drawn with replacement): S[k*s + j] for every batch k of epoch e. */
void or_negatives(int64_t n, int64_t nbatches, int32_t s, uint64_t seed, uint32_t epoch,
                  int32_t *S)
{
    for (int64_t k = 0; k < nbatches; ++k)
        for (int32_t j = 0; j < s; ++j) {
            uint32_t out[4];
            philox_call(seed, epoch, (uint32_t)k, (uint32_t)j, TAG_NEG, out);
            S[k * s + j] = (int32_t)or_uniform_index(out[0], out[1], n);
        }
}

/* Fixed evaluation negatives of the loss: W[u*s + j]. */
void or_eval_negatives(int64_t n, int32_t s, uint64_t seed, int32_t *W)
{
    for (int64_t u = 0; u < n; ++u)
        for (int32_t j = 0; j < s; ++j) {
            uint32_t out[4];
            philox_call(seed, (uint32_t)u, (uint32_t)((uint64_t)u >> 32), (uint32_t)j, TAG_EVAL, out);
            W[u * s + j] = (int32_t)or_uniform_index(out[0], out[1], n);
        }
}

/* Random-walk neighbourhood of u in epoch e (Algorithm 3): starting at u, each
 * step moves to a uniformly chosen neighbour of the current vertex (step i
 * draws Philox(e, u, i, TAG_WALK) and takes the neighbour at that uniform
 * index of the current row); a vertex not yet in the set joins it (u itself
 * included, if the walk comes back to it).  The paper's loop runs until the
 * set holds k vertices, which never happens when fewer than k vertices are
 * reachable, so the walk also stops after 4k steps or at a vertex with no
 * neighbours.  list receives the set in the order its vertices were first
 * reached; raw (may be NULL, room for 4k) every step's vertex, *nraw their
 * number.  Returns the size of the set. */
int32_t or_walk(const int64_t *rowptr, const int32_t *colidx, uint64_t seed, uint32_t epoch, int64_t u,
                int32_t k, int32_t *list, int32_t *raw, int32_t *nraw)
{
    int32_t len = 0, steps = 0;
    int64_t w = u;
    while (len < k && steps < 4 * k) {
        int64_t deg = rowptr[w + 1] - rowptr[w];
        if (deg == 0) break;
        uint32_t out[4];
        philox_call(seed, epoch, (uint32_t)u, (uint32_t)steps, TAG_WALK, out);
        int32_t next = colidx[rowptr[w] + or_uniform_index(out[0], out[1], deg)];
        if (raw) raw[steps] = next;
        ++steps;
        int seen = 0;
        for (int32_t j = 0; j < len && !seen; ++j) seen = list[j] == next;
        if (!seen) list[len++] = next;
        w = next;
    }
    if (nraw) *nraw = steps;
    return len;
}

/* ------------------------------------------------------------------------ */
/* Per-pair forces (gradients of the per-vertex loss with respect to z_u, the
 * other row held fixed).  a = z_u, c = the other row.  Accumulated into g. */

double or_bf16_round(double x)
{
    /* round a double to the nearest bfloat16 (8 significant bits), ties to even */
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    double m = frexp(x, &e);           /* x = m * 2^e, 0.5 <= |m| < 1 */
    double scaled = ldexp(m, 8);       /* 8 significant bits left of the point */
    double r = nearbyint(scaled);      /* default rounding mode: to nearest even */
    return ldexp(r, e - 8);
}

static inline double input(const double *row, int i, int emul)
{
    return emul ? or_bf16_round(row[i]) : row[i];
}

static double sigmoid(double x)
{
    if (x >= 0) return 1.0 / (1.0 + exp(-x));
    double ex = exp(x);
    return ex / (1.0 + ex);
}

/* Magnitude, along the unit vector (a-c)/t, of the attractive gradient of the
 * Table 2 models at distance t = |a - c|, the pull written as a positive
 * gradient: t^2 (Fruchterman-Reingold), log(1 + t) (LinLog), t (ForceAtlas). */
static double attraction_magnitude(int force, double t)
{
    switch (force) {
    case OR_FR: return t * t;
    case OR_LINLOG: return log1p(t);
    default: return t; /* OR_FORCEATLAS */
    }
}

/* Attractive force: sigmoid Eq. 5 term, (sigma(a.c) - 1) c; the distance-based
 * models: magnitude times the unit vector (a-c)/t (0 when t = 0, where every
 * magnitude above vanishes faster than t, except LinLog's, whose ratio
 * log(1 + t)/t tends to 1: its limit is taken). */
static void add_attraction(int d, int force, const double *a, const double *c, double *g,
                           int emul)
{
    if (force == OR_SIGMOID) {
        double x = 0.0;
        for (int i = 0; i < d; ++i) x += input(a, i, emul) * input(c, i, emul);
        double coef = -sigmoid(-x); /* sigma(x) - 1 */
        for (int i = 0; i < d; ++i) g[i] += coef * input(c, i, emul);
    } else {
        double q = 0.0;
        for (int i = 0; i < d; ++i) {
            double df = input(a, i, emul) - input(c, i, emul);
            q += df * df;
        }
        double coef;
        if (force == OR_STUDENT_T) {
            coef = 2.0 / (1.0 + q); /* Eq. 8, 2t/(1+t^2), times 1/t */
        } else {
            double t = sqrt(q);
            coef = t > 0.0 ? attraction_magnitude(force, t) / t : (force == OR_LINLOG ? 1.0 : 0.0);
        }
        for (int i = 0; i < d; ++i) g[i] += coef * (input(a, i, emul) - input(c, i, emul));
    }
}

/* Repulsive force: sigmoid Eq. 6 term, sigma(a.c) c; Student-t Eq. 9 term
 * times (a-c)/t, regularised: the gradient of log(1+q) - log(q+eps),
 * -2 (1-eps) (a-c) / ((q+eps)(1+q)); with eps = 0 it is the paper's formula
 * and is taken as 0 when q = 0. */
static void add_repulsion(int d, int force, double eps, const double *a, const double *c,
                          double *g, int emul)
{
    if (force == OR_SIGMOID) {
        double x = 0.0;
        for (int i = 0; i < d; ++i) x += input(a, i, emul) * input(c, i, emul);
        double coef = sigmoid(x);
        for (int i = 0; i < d; ++i) g[i] += coef * input(c, i, emul);
    } else {
        double q = 0.0;
        for (int i = 0; i < d; ++i) {
            double df = input(a, i, emul) - input(c, i, emul);
            q += df * df;
        }
        if (q + eps == 0.0) return;
        double coef;
        if (force == OR_STUDENT_T) {
            coef = -2.0 * (1.0 - eps) / ((q + eps) * (1.0 + q));
        } else {
            /* Table 2: magnitude 1/t pushing away, times (a-c)/t: -(a-c)/t^2,
             * regularised as -(a-c)/(q+eps), the gradient of -log(q+eps)/2 */
            coef = -1.0 / (q + eps);
        }
        for (int i = 0; i < d; ++i) g[i] += coef * (input(a, i, emul) - input(c, i, emul));
    }
}

/* Gradient of L(u) (Eq. 2) for one vertex, given its row, its neighbour rows
 * and its negative rows (Algorithm 2, body of the parallel loop). */
void or_vertex_gradient(int d, int force, double eps, const double *zu,
                        int32_t nnbr, const double *nbr_rows, int32_t nneg,
                        const double *neg_rows, int emul, double *g)
{
    for (int i = 0; i < d; ++i) g[i] = 0.0;
    for (int32_t j = 0; j < nnbr; ++j) add_attraction(d, force, zu, nbr_rows + (size_t)j * d, g, emul);
    for (int32_t j = 0; j < nneg; ++j) add_repulsion(d, force, eps, zu, neg_rows + (size_t)j * d, g, emul);
}

/* ------------------------------------------------------------------------ */
/* Per-pair loss terms of Eq. 2: -log delta for a neighbour, -log(1 - delta)
 * for a negative.  Sigmoid (Eq. 3): softplus(-x), softplus(x).  Student-t
 * (Eq. 7): log(1+q), log(1+q) - log(q+eps). */

static double softplus(double y)
{
    return (y > 0 ? y : 0.0) + log1p(exp(-fabs(y)));
}

/* The Table 2 models have no likelihood in the paper; their loss is the
 * potential whose gradient the forces above are: attraction t^3/3 (FR),
 * (1 + t) log(1 + t) - t (LinLog), t^2/2 (ForceAtlas); repulsion
 * -log(q + eps)/2, taken as 0 where q + eps = 0 (as the force is). */
double or_pair_loss(int d, int force, double eps, const double *a, const double *c,
                    int repulsive, int emul)
{
    if (force == OR_SIGMOID) {
        double x = 0.0;
        for (int i = 0; i < d; ++i) x += input(a, i, emul) * input(c, i, emul);
        return repulsive ? softplus(x) : softplus(-x);
    }
    double q = 0.0;
    for (int i = 0; i < d; ++i) {
        double df = input(a, i, emul) - input(c, i, emul);
        q += df * df;
    }
    if (force == OR_STUDENT_T) return repulsive ? log1p(q) - log(q + eps) : log1p(q);
    if (repulsive) return q + eps == 0.0 ? 0.0 : -0.5 * log(q + eps);
    double t = sqrt(q);
    if (force == OR_FR) return t * t * t / 3.0;
    if (force == OR_LINLOG) return (1.0 + t) * log1p(t) - t;
    return 0.5 * q; /* OR_FORCEATLAS */
}

/* Loss of Eq. 2 summed over all vertices, with W[u*s+j] as the negatives of
 * u.  out[0] = total, out[1] = attractive part, out[2] = repulsive part. */
void or_loss(int64_t n, int32_t d, const int64_t *rowptr, const int32_t *colidx,
             const double *Z, int32_t s, const int32_t *W, int force, double eps,
             int emul, int nthreads, double out[3])
{
    double *ra = (double *)malloc(sizeof(double) * (size_t)n);
    double *rr = (double *)malloc(sizeof(double) * (size_t)n);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t u = 0; u < n; ++u) {
        const double *zu = Z + (size_t)u * d;
        double la = 0.0, lr = 0.0;
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
            la += or_pair_loss(d, force, eps, zu, Z + (size_t)colidx[e] * d, 0, emul);
        for (int32_t j = 0; j < s; ++j)
            lr += or_pair_loss(d, force, eps, zu, Z + (size_t)W[u * s + j] * d, 1, emul);
        ra[u] = la;
        rr[u] = lr;
    }
    double sa = 0.0, sr = 0.0;
    for (int64_t u = 0; u < n; ++u) { sa += ra[u]; sr += rr[u]; }
    free(ra);
    free(rr);
    out[0] = sa + sr;
    out[1] = sa;
    out[2] = sr;
}

/* ------------------------------------------------------------------------ */
/* One epoch of Algorithm 1.
 *
 *   Z        : n x d FP64 state, updated in place
 *   b, s     : batch size, negatives per batch
 *   lr       : step size of this epoch
 *   perm_mode: 0 keyed random partition, 1 identity
 *   S_inject : if non-NULL, the negatives to use (nbatches*s entries) instead
 *              of the Philox draw (used by relabelling tests)
 *   pairs    : if non-NULL, receives the number of pair evaluations
 *   k_begin, k_end : run only batches [k_begin, k_end) (a bounded sample of the
 *              epoch for timing); pass 0, -1 for the whole epoch.
 *   walk_k   : 0: N(u) is u's row of the graph; k > 0: N(u) is the random-walk
 *              neighbourhood of Algorithm 3 (or_walk) with walks of length k.
 *
 * Within a batch every gradient reads the batch-start state (Algorithm 2 reads
 * Z, Algorithm 1 applies the step after GradMinibatch returns); only the batch
 * vertices are updated (Eq. 10). */
int or_epoch(int64_t n, int32_t d, const int64_t *rowptr, const int32_t *colidx,
             double *Z, int32_t b, int32_t s, int force, double eps, double lr,
             uint64_t seed, uint32_t epoch, int perm_mode, const int32_t *S_inject,
             int emul, int nthreads, int64_t *pairs, int64_t k_begin, int64_t k_end,
             int32_t walk_k)
{
    if (n <= 0 || d <= 0 || b <= 0 || s < 0) return 1;
    int64_t nb = (n + b - 1) / b;
    if (k_end < 0 || k_end > nb) k_end = nb;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s > 0 ? s : 1));
    double *G = (double *)malloc(sizeof(double) * (size_t)b * d);
    int32_t *WL = (int32_t *)malloc(sizeof(int32_t) * (size_t)b * (walk_k > 0 ? walk_k : 1));
    int32_t *WN = (int32_t *)malloc(sizeof(int32_t) * (size_t)b);
    if (!perm || !S || !G || !WL || !WN) { free(perm); free(S); free(G); free(WL); free(WN); return 2; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    or_partition(n, seed, epoch, perm_mode, perm);
    int64_t npairs = 0;
    for (int64_t k = k_begin; k < k_end; ++k) {
        int64_t lo = k * b, hi = lo + b < n ? lo + b : n;
        for (int32_t j = 0; j < s; ++j) {
            if (S_inject) {
                S[j] = S_inject[k * s + j];
            } else {
                uint32_t out[4];
                philox_call(seed, epoch, (uint32_t)k, (uint32_t)j, TAG_NEG, out);
                S[j] = (int32_t)or_uniform_index(out[0], out[1], n);
            }
        }
        /* GradMinibatch: every vertex of the batch independently */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
        for (int64_t p = lo; p < hi; ++p) {
            int64_t u = perm[p];
            const double *zu = Z + (size_t)u * d;
            double *g = G + (size_t)(p - lo) * d;
            for (int i = 0; i < d; ++i) g[i] = 0.0;
            if (walk_k > 0) {
                int32_t *list = WL + (size_t)(p - lo) * walk_k;
                WN[p - lo] = or_walk(rowptr, colidx, seed, epoch, u, walk_k, list, NULL, NULL);
                for (int32_t j = 0; j < WN[p - lo]; ++j)
                    add_attraction(d, force, zu, Z + (size_t)list[j] * d, g, emul);
            } else {
                for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
                    add_attraction(d, force, zu, Z + (size_t)colidx[e] * d, g, emul);
            }
            for (int32_t j = 0; j < s; ++j)
                add_repulsion(d, force, eps, zu, Z + (size_t)S[j] * d, g, emul);
        }
        /* the update of Eq. 10 for the batch vertices */
        for (int64_t p = lo; p < hi; ++p) {
            int64_t u = perm[p];
            double *zu = Z + (size_t)u * d;
            const double *g = G + (size_t)(p - lo) * d;
            for (int i = 0; i < d; ++i) zu[i] -= lr * g[i];
            npairs += (walk_k > 0 ? WN[p - lo] : rowptr[u + 1] - rowptr[u]) + s;
        }
    }
    if (pairs) *pairs = npairs;
    free(perm);
    free(S);
    free(G);
    free(WL);
    free(WN);
    return 0;
}

/* Step size of epoch e: constant, or decaying linearly to zero over
 * total_epochs (the paper fixes only the initial value, Algorithm 1). */
double or_learning_rate(double lr0, int schedule, int32_t epoch, int32_t total_epochs)
{
    if (schedule == 1 && total_epochs > 0) return lr0 * (1.0 - (double)epoch / (double)total_epochs);
    return lr0;
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
