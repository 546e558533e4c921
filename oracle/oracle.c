/*
 * CPU oracle for BANG's batched PQ greedy search (arXiv 2401.11324).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or constant with the GPU
 * path.  Plain, slow and sequential by design: every routine follows the
 * paper's definition step by step, with no blocking, fusion or reordering
 * beyond what the definition states.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (see build.py).
 * -ffp-contract=off matters: the FP32 table and ADC sums below are the
 * canonical rounding sequence that the GPU path must reproduce bit for bit.
 *
 * Arithmetic conventions (the reading of the paper this oracle encodes):
 *  - distances are squared Euclidean everywhere (the PQ table section builds
 *    squared distances; ranking is identical to the plain Euclidean one);
 *  - PQ distance table (section "Construction of PQDistTable in Parallel"):
 *      T[j][c] = sum_{t < d/m} (q[j*d/m + t] - cb[j][c][t])^2
 *    summed left to right in FP32, one rounding per subtraction, product and
 *    addition;
 *  - asymmetric distance (section "Parallel Neighbour Distance
 *    Computation"): ADC(x) = sum_{j < m} T[j][code_x[j]], left to right in
 *    FP32;
 *  - exact re-rank distance (section "Re-ranking"): integer data uses an
 *    exact integer sum converted once to FP32; float data uses the same
 *    left-to-right FP32 form as the table;
 *  - every ordering is by (distance, node id): ids break distance ties.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_F32 0
#define OR_U8 1
#define OR_I8 2
#define OR_F64 3
#define OR_NONE 0xFFFFFFFFu

/* Index as handed over by the Python wrapper (all host memory). */
typedef struct {
  uint64_t n;
  uint32_t d;
  int32_t dtype;          /* OR_F32 / OR_U8 / OR_I8 */
  const void* base;       /* n*d elements */
  uint32_t R;
  const uint32_t* adj;    /* n*R, OR_NONE marks an empty slot */
  uint32_t medoid;
  uint32_t m;
  const float* codebooks; /* m*256*(d/m) */
  const uint8_t* codes;   /* n*m */
} or_index;

static double elem_d(const void* p, int dt, uint64_t i) {
  switch (dt) {
    case OR_F32: return (double)((const float*)p)[i];
    case OR_U8: return (double)((const uint8_t*)p)[i];
    case OR_I8: return (double)((const int8_t*)p)[i];
    default: return ((const double*)p)[i];
  }
}

/* Query element as FP32.  Integer elements convert exactly. */
static float elem_f(const void* p, int dt, uint64_t i) {
  switch (dt) {
    case OR_F32: return ((const float*)p)[i];
    case OR_U8: return (float)((const uint8_t*)p)[i];
    case OR_I8: return (float)((const int8_t*)p)[i];
    default: return (float)((const double*)p)[i];
  }
}

/* ------------------------------------------------------------------------
 * Stage 1: PQ distance table (section "Construction of PQDistTable in
 * Parallel").  One query, all m subspaces, all 256 centroids.
 * ---------------------------------------------------------------------- */
static void pq_table_one(const void* q, int qdt, uint32_t d, const float* cb,
                         uint32_t m, float* T) {
  uint32_t ds = d / m;
  for (uint32_t j = 0; j < m; ++j) {
    for (uint32_t c = 0; c < 256; ++c) {
      const float* cent = cb + ((uint64_t)j * 256 + c) * ds;
      float acc = 0.0f;
      for (uint32_t t = 0; t < ds; ++t) {
        float diff = elem_f(q, qdt, (uint64_t)j * ds + t) - cent[t];
        float sq = diff * diff;
        acc = acc + sq;
      }
      T[(uint64_t)j * 256 + c] = acc;
    }
  }
}

void or_pq_tables(const void* queries, int qdt, uint64_t nq, uint32_t d,
                  const float* cb, uint32_t m, float* T, int nthreads) {
  int64_t i;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (i = 0; i < (int64_t)nq; ++i) {
    const char* qp = (const char*)queries;
    size_t esz = (qdt == OR_F32) ? 4 : (qdt == OR_F64 ? 8 : 1);
    pq_table_one(qp + (size_t)i * d * esz, qdt, d, cb, m,
                 T + (uint64_t)i * m * 256);
  }
}

/* Asymmetric distance of one compressed vector against a query's table. */
static float adc_one(const float* T, const uint8_t* code, uint32_t m) {
  float acc = 0.0f;
  for (uint32_t j = 0; j < m; ++j) acc = acc + T[(uint64_t)j * 256 + code[j]];
  return acc;
}

/* ------------------------------------------------------------------------
 * Reduced-precision table storage (the precision form).  Both forms are
 * derived from the canonical FP32 table of the query, so they are fully
 * determined by it:
 *  - F16: every entry times a power-of-two scale 2^-k (the smallest k >= 0
 *    that brings the largest entry to <= 65504, the largest half value),
 *    rounded to the nearest half-precision value, ties to even.  ADC sums
 *    the half values, widened to FP32, left to right in FP32.
 *  - U8: per subspace j the offset lo_j = min_c T[j][c]; one scale for the
 *    query, inv = 255 / max_j (max_c T[j][c] - lo_j) in FP32 (0 if every
 *    range is 0); entry = rint((T[j][c] - lo_j) * inv), ties to even, in
 *    [0, 255].  ADC is the exact integer sum of the m entries; the constant
 *    sum of the offsets and the common scale do not change any order, so
 *    the sum itself (converted to FP32, exact below 2^24) is the distance
 *    the search ranks by.
 * ---------------------------------------------------------------------- */
#define OR_TABLE_F32 0
#define OR_TABLE_F16 1
#define OR_TABLE_U8 2
/* No table at all: the paper's Exact-distance Version (section
 * "Implementation Variants").  The search ranks every node by its exact
 * distance to the query (the re-rank's distance), and there is no re-rank:
 * the answer is the k first entries of the final worklist. */
#define OR_TABLE_EXACT 3

/* FP32 -> IEEE half, round to nearest, ties to even (finite inputs). */
uint16_t or_f32_to_f16(float f) {
  uint32_t x;
  memcpy(&x, &f, 4);
  uint32_t sign = (x >> 16) & 0x8000u;
  uint32_t ax = x & 0x7FFFFFFFu;
  if (ax >= 0x477FF000u) return (uint16_t)(sign | 0x7C00u); /* >= 65520: inf */
  if (ax >= 0x38800000u) {                                   /* half normal */
    uint32_t h = ((((ax >> 23) - 127 + 15) << 10) | ((ax >> 13) & 0x3FFu));
    uint32_t rem = ax & 0x1FFFu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;
    return (uint16_t)(sign | h);
  }
  /* half subnormal: units of 2^-24, rounded to nearest even (exact in
   * double: the scaled value has at most 24 significant bits) */
  double q = (double)fabsf(f) * 16777216.0;
  double n = rint(q);
  return (uint16_t)(sign | (uint32_t)n);
}

float or_f16_to_f32(uint16_t h) {
  uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  uint32_t e = (h >> 10) & 0x1Fu, mant = h & 0x3FFu;
  float v;
  if (e == 0)
    v = (float)mant * 5.9604644775390625e-8f; /* mant * 2^-24, exact */
  else if (e == 31)
    v = mant ? NAN : INFINITY;
  else {
    uint32_t b = ((e - 15 + 127) << 23) | (mant << 13);
    memcpy(&v, &b, 4);
  }
  uint32_t vb;
  memcpy(&vb, &v, 4);
  vb |= sign;
  memcpy(&v, &vb, 4);
  return v;
}

typedef struct {
  int mode;
  uint32_t m;
  const float* T32; /* canonical table (built for every mode but EXACT) */
  uint16_t* T16;
  uint8_t* T8;
  const void* q;    /* the query (EXACT) */
} qtable;

static void quantize_table(qtable* t) {
  uint64_t ne = (uint64_t)t->m * 256;
  if (t->mode == OR_TABLE_F16) {
    float mx = 0.0f;
    for (uint64_t i = 0; i < ne; ++i)
      if (t->T32[i] > mx) mx = t->T32[i];
    float s = 1.0f;
    while (mx * s > 65504.0f) s = s * 0.5f;
    for (uint64_t i = 0; i < ne; ++i) t->T16[i] = or_f32_to_f16(t->T32[i] * s);
  } else if (t->mode == OR_TABLE_U8) {
    float R = 0.0f;
    for (uint32_t j = 0; j < t->m; ++j) {
      float lo = t->T32[(uint64_t)j * 256], hi = lo;
      for (uint32_t c = 1; c < 256; ++c) {
        float v = t->T32[(uint64_t)j * 256 + c];
        if (v < lo) lo = v;
        if (v > hi) hi = v;
      }
      float range = hi - lo;
      if (range > R) R = range;
    }
    float inv = R > 0.0f ? 255.0f / R : 0.0f;
    for (uint32_t j = 0; j < t->m; ++j) {
      float lo = t->T32[(uint64_t)j * 256];
      for (uint32_t c = 1; c < 256; ++c)
        if (t->T32[(uint64_t)j * 256 + c] < lo) lo = t->T32[(uint64_t)j * 256 + c];
      for (uint32_t c = 0; c < 256; ++c) {
        float diff = t->T32[(uint64_t)j * 256 + c] - lo;
        float v = rintf(diff * inv);
        t->T8[(uint64_t)j * 256 + c] = (uint8_t)(v > 255.0f ? 255.0f : v);
      }
    }
  }
}

/* Distance the search ranks by, for the table's storage form. */
static float adc_q(const qtable* t, const uint8_t* code) {
  if (t->mode == OR_TABLE_F32) return adc_one(t->T32, code, t->m);
  if (t->mode == OR_TABLE_F16) {
    float acc = 0.0f;
    for (uint32_t j = 0; j < t->m; ++j)
      acc = acc + or_f16_to_f32(t->T16[(uint64_t)j * 256 + code[j]]);
    return acc;
  }
  uint32_t acc = 0;
  for (uint32_t j = 0; j < t->m; ++j) acc += t->T8[(uint64_t)j * 256 + code[j]];
  return (float)acc;
}

/* Quantised tables of a batch (for tests): out16 [nq][m][256] or out8. */
void or_quantize_tables(const float* T, uint64_t nq, uint32_t m, int mode,
                        uint16_t* out16, uint8_t* out8) {
  for (uint64_t q = 0; q < nq; ++q) {
    qtable t = {mode, m, T + q * m * 256, out16 ? out16 + q * m * 256 : NULL,
                out8 ? out8 + q * m * 256 : NULL, NULL};
    quantize_table(&t);
  }
}

void or_adc(const float* T, const uint8_t* codes, uint32_t m,
            const uint32_t* ids, uint64_t cnt, float* out) {
  for (uint64_t i = 0; i < cnt; ++i)
    out[i] = adc_one(T, codes + (uint64_t)ids[i] * m, m);
}

/* ------------------------------------------------------------------------
 * Exact distance used by the re-rank (section "Re-ranking").
 * ---------------------------------------------------------------------- */
static float exact_dist(const or_index* ix, const void* q, uint32_t id) {
  uint32_t d = ix->d;
  if (ix->dtype == OR_F32) {
    const float* x = (const float*)ix->base + (uint64_t)id * d;
    const float* qq = (const float*)q;
    float acc = 0.0f;
    for (uint32_t t = 0; t < d; ++t) {
      float diff = x[t] - qq[t];
      float sq = diff * diff;
      acc = acc + sq;
    }
    return acc;
  }
  int64_t acc = 0;
  for (uint32_t t = 0; t < d; ++t) {
    int64_t a = (ix->dtype == OR_U8)
                    ? (int64_t)((const uint8_t*)ix->base)[(uint64_t)id * d + t]
                    : (int64_t)((const int8_t*)ix->base)[(uint64_t)id * d + t];
    int64_t b = (ix->dtype == OR_U8) ? (int64_t)((const uint8_t*)q)[t]
                                     : (int64_t)((const int8_t*)q)[t];
    acc += (a - b) * (a - b);
  }
  return (float)acc;
}

/* The distance the search ranks node x by: its PQ distance from the table,
 * or, without a table, its exact distance. */
static float node_dist(const or_index* ix, const qtable* T, uint32_t x) {
  if (T->mode == OR_TABLE_EXACT) return exact_dist(ix, T->q, x);
  return adc_q(T, ix->codes + (uint64_t)x * ix->m);
}

/* ------------------------------------------------------------------------
 * Stage 2: greedy search (Algorithm 1, with the PQ distance of Algorithm 2
 * as the distance to the query).
 * ---------------------------------------------------------------------- */
typedef struct {
  float dist;
  uint32_t id;
  int32_t visited;
} entry;

static int entry_cmp(const void* a, const void* b) {
  const entry* x = (const entry*)a;
  const entry* y = (const entry*)b;
  if (x->dist < y->dist) return -1;
  if (x->dist > y->dist) return 1;
  if (x->id < y->id) return -1;
  if (x->id > y->id) return 1;
  return 0;
}

/*
 * The paper's visited filter (section "Parallel Filtering of Visited
 * Neighbours"; parameters in section "Algorithm Parameters"): one array of
 * z = 399,887 boolean entries per query and two FNV-1a hash functions.
 * FNV-1a-32 is the published one (offset basis 2166136261, prime 16777619:
 * for each byte, xor it in, then multiply).  The paper does not say how its
 * two functions differ; read here as the same function over the id's four
 * little-endian bytes with two offset bases, the standard one and the
 * standard one xor 0xA5A5A5A5, each taken mod z.
 */
#define OR_BLOOM_Z 399887u
#define OR_FNV_BASIS 0x811C9DC5u
#define OR_FNV_PRIME 0x01000193u
#define OR_BLOOM_SALT 0xA5A5A5A5u

uint32_t or_fnv1a32(const uint8_t* p, uint64_t n, uint32_t basis) {
  uint32_t h = basis;
  for (uint64_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= OR_FNV_PRIME;
  }
  return h;
}

/* The two entries of node x. */
void or_bloom_slots(uint32_t x, uint32_t* h1, uint32_t* h2) {
  uint8_t b[4] = {(uint8_t)x, (uint8_t)(x >> 8), (uint8_t)(x >> 16),
                  (uint8_t)(x >> 24)};
  *h1 = or_fnv1a32(b, 4, OR_FNV_BASIS) % OR_BLOOM_Z;
  *h2 = or_fnv1a32(b, 4, OR_FNV_BASIS ^ OR_BLOOM_SALT) % OR_BLOOM_Z;
}

/* Algorithm 2's GetBloomFilter followed, when it fails, by SetBloomFilter:
 * returns 1 when both entries of x are already set (x counts as visited),
 * else sets both and returns 0. */
static int bloom_test_and_set(uint8_t* bf, uint32_t x) {
  uint32_t h1, h2;
  or_bloom_slots(x, &h1, &h2);
  if (bf[h1] && bf[h2]) return 1;
  bf[h1] = 1;
  bf[h2] = 1;
  return 0;
}

/* Per-query results of stage 2. */
typedef struct {
  uint32_t iters;  /* I = number of expanded nodes = |C| */
  uint32_t status; /* 1 if the iteration cap stopped the search */
  uint64_t added;  /* distances computed for nodes new to the worklist */
} or_counters;

/*
 * mode 0: Algorithm 1 as printed.  The worklist is a set of nodes: the
 *         union with adj(u*) skips nodes already in it, then the worklist
 *         keeps its t nearest entries.
 * mode 1: the filtered form of Algorithm 2: a node's distance is computed
 *         only the first time it is seen (an exact seen-set replaces the
 *         paper's Bloom filter), the new nodes are sorted and merged into
 *         the worklist, which keeps its t nearest entries.
 * Both modes expand the same nodes in the same order and end with the same
 * worklist; the tests check that.
 * mode 2: Algorithm 2 with the paper's Bloom filter in place of the exact
 *         seen-set: the neighbours of u* are tested and set one after the
 *         other in stored order, so a neighbour sees the entries set by the
 *         ones before it in the same row.  A false positive drops a node
 *         that was never seen; nothing seen is ever kept.
 *
 * On return C[0..iters) holds the expanded nodes with their PQ distances in
 * expansion order, and Lout[0..*Llen) the final worklist.
 */
static void greedy_search(const or_index* ix, const qtable* T, uint32_t Lcap,
                          uint32_t iter_cap, int mode, uint32_t* seen,
                          uint32_t stamp, uint8_t* bloom, entry* L,
                          uint32_t* Llen, entry* C, entry* scratch,
                          or_counters* cnt) {
  uint32_t R = ix->R;
  uint32_t s = ix->medoid;
  uint32_t len = 1;
  L[0].dist = node_dist(ix, T, s);
  L[0].id = s;
  L[0].visited = 0;
  if (mode == 1) seen[s] = stamp;
  if (mode == 2) {
    memset(bloom, 0, OR_BLOOM_Z);
    bloom_test_and_set(bloom, s);
  }
  cnt->iters = 0;
  cnt->status = 0;
  cnt->added = 0;
  for (;;) {
    /* u* = arg min over L \ V: L is kept sorted, so the first unvisited. */
    int64_t pos = -1;
    for (uint32_t i = 0; i < len; ++i)
      if (!L[i].visited) {
        pos = i;
        break;
      }
    if (pos < 0) break; /* L \ V is empty: converged */
    if (cnt->iters == iter_cap) {
      cnt->status = 1;
      break;
    }
    L[pos].visited = 1; /* V <- V u {u*} */
    C[cnt->iters++] = L[pos];
    uint32_t u = L[pos].id;
    const uint32_t* nb = ix->adj + (uint64_t)u * R;
    if (mode == 0) {
      /* L <- L u adj(u*) */
      for (uint32_t r = 0; r < R; ++r) {
        uint32_t x = nb[r];
        if (x == OR_NONE) continue;
        int present = 0;
        for (uint32_t i = 0; i < len; ++i)
          if (L[i].id == x) {
            present = 1;
            break;
          }
        if (present) continue;
        L[len].dist = node_dist(ix, T, x);
        L[len].id = x;
        L[len].visited = 0;
        ++len;
        cnt->added++;
      }
      /* keep up to t nearest */
      qsort(L, len, sizeof(entry), entry_cmp);
      if (len > Lcap) len = Lcap;
    } else {
      /* filter: N' = neighbours not seen before */
      uint32_t np = 0;
      for (uint32_t r = 0; r < R; ++r) {
        uint32_t x = nb[r];
        if (x == OR_NONE) continue;
        if (mode == 2) {
          if (bloom_test_and_set(bloom, x)) continue;
        } else {
          if (seen[x] == stamp) continue;
          seen[x] = stamp;
        }
        scratch[np].dist = node_dist(ix, T, x);
        scratch[np].id = x;
        scratch[np].visited = 0;
        ++np;
      }
      cnt->added += np;
      /* sort N', then merge it into L keeping the t nearest */
      qsort(scratch, np, sizeof(entry), entry_cmp);
      entry* merged = scratch + R;
      uint32_t a = 0, b = 0, o = 0;
      while (o < Lcap && (a < len || b < np)) {
        if (b >= np || (a < len && entry_cmp(&L[a], &scratch[b]) < 0))
          merged[o++] = L[a++];
        else
          merged[o++] = scratch[b++];
      }
      memcpy(L, merged, o * sizeof(entry));
      len = o;
    }
  }
  *Llen = len;
}

/* Stage 3: re-rank.  Candidates are the expanded nodes; when there are more
 * than c_max of them, the c_max nearest by (PQ distance, id) are kept. */
static void rerank_entries(const or_index* ix, const void* q, entry* C,
                           uint32_t nc, uint32_t c_max, uint32_t k,
                           uint32_t* out_ids, float* out_d) {
  if (nc > c_max) {
    qsort(C, nc, sizeof(entry), entry_cmp);
    nc = c_max;
  }
  for (uint32_t i = 0; i < nc; ++i) {
    C[i].dist = exact_dist(ix, q, C[i].id);
    C[i].visited = 0;
  }
  qsort(C, nc, sizeof(entry), entry_cmp);
  for (uint32_t i = 0; i < k; ++i) {
    if (i < nc) {
      out_ids[i] = C[i].id;
      out_d[i] = C[i].dist;
    } else {
      out_ids[i] = OR_NONE;
      out_d[i] = INFINITY;
    }
  }
}

static size_t dt_size(int dt) {
  return dt == OR_F32 ? 4 : (dt == OR_F64 ? 8 : 1);
}

/*
 * Whole path for a batch: table -> greedy search -> re-rank.
 * Outputs (each may be NULL except ids/dists):
 *   ids[nq][k], dists[nq][k]      re-ranked result, padded (OR_NONE, +inf)
 *   pq_ids[nq][k], pq_dists[nq][k] Algorithm 1's own answer: the k nearest
 *                                 entries of the final worklist (PQ order)
 *   cand[nq][cand_cap]            expanded nodes in expansion order, padded
 *   counters[nq][4]               {I, status, added_lo, added_hi}
 */
int or_search(const or_index* ix, const void* queries, uint64_t nq, uint32_t k,
              uint32_t Lcap, uint32_t c_max, uint32_t iter_cap, int mode,
              int table_mode,
              uint32_t* ids, float* dists, uint32_t* pq_ids, float* pq_dists,
              uint32_t* cand, uint32_t cand_cap, uint32_t* counters,
              int nthreads) {
  if (k == 0 || Lcap < k || ix->d % ix->m != 0 || mode < 0 || mode > 2)
    return -1;
  int64_t qi;
  int bad = 0;
#pragma omp parallel num_threads(nthreads)
  {
    float* T = (float*)malloc((size_t)ix->m * 256 * sizeof(float));
    uint16_t* T16 = (uint16_t*)malloc((size_t)ix->m * 256 * sizeof(uint16_t));
    uint8_t* T8 = (uint8_t*)malloc((size_t)ix->m * 256);
    entry* L = (entry*)malloc((size_t)(Lcap + ix->R) * sizeof(entry));
    entry* C = (entry*)malloc((size_t)(iter_cap + 1) * sizeof(entry));
    entry* scr = (entry*)malloc((size_t)(2 * ix->R + Lcap) * sizeof(entry));
    uint32_t* seen = (uint32_t*)calloc(ix->n, sizeof(uint32_t));
    uint8_t* bloom = mode == 2 ? (uint8_t*)malloc(OR_BLOOM_Z) : NULL;
    uint32_t stamp = 0;
    if (!T || !T16 || !T8 || !L || !C || !scr || !seen ||
        (mode == 2 && !bloom)) {
#pragma omp atomic write
      bad = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (qi = 0; qi < (int64_t)nq; ++qi) {
        const char* q = (const char*)queries + (size_t)qi * ix->d * dt_size(ix->dtype);
        if (table_mode != OR_TABLE_EXACT)
          pq_table_one(q, ix->dtype, ix->d, ix->codebooks, ix->m, T);
        qtable qt = {table_mode, ix->m, T, T16, T8, q};
        quantize_table(&qt);
        or_counters cn;
        uint32_t Llen;
        ++stamp;
        greedy_search(ix, &qt, Lcap, iter_cap, mode, seen, stamp, bloom, L,
                      &Llen, C, scr, &cn);
        if (pq_ids)
          for (uint32_t i = 0; i < k; ++i) {
            pq_ids[qi * k + i] = i < Llen ? L[i].id : OR_NONE;
            pq_dists[qi * k + i] = i < Llen ? L[i].dist : INFINITY;
          }
        if (cand)
          for (uint32_t i = 0; i < cand_cap; ++i)
            cand[qi * cand_cap + i] = i < cn.iters ? C[i].id : OR_NONE;
        if (counters) {
          counters[qi * 4 + 0] = cn.iters;
          counters[qi * 4 + 1] = cn.status;
          counters[qi * 4 + 2] = (uint32_t)(cn.added & 0xFFFFFFFFu);
          counters[qi * 4 + 3] = (uint32_t)(cn.added >> 32);
        }
        if (table_mode == OR_TABLE_EXACT) {
          /* no re-rank: the worklist already holds exact distances */
          for (uint32_t i = 0; i < k; ++i) {
            ids[qi * k + i] = i < Llen ? L[i].id : OR_NONE;
            dists[qi * k + i] = i < Llen ? L[i].dist : INFINITY;
          }
        } else {
          rerank_entries(ix, q, C, cn.iters, c_max, k, ids + qi * k,
                         dists + qi * k);
        }
      }
    }
    free(T);
    free(T16);
    free(T8);
    free(L);
    free(C);
    free(scr);
    free(seen);
    free(bloom);
  }
  return bad ? -2 : 0;
}

/* Stage 3 alone: exact top-k over a given candidate list per query.  Ids
 * equal to OR_NONE or >= n are padding and are skipped. */
int or_rerank(const or_index* ix, const void* queries, uint64_t nq,
              const uint32_t* cand, uint32_t c_max, uint32_t k, uint32_t* ids,
              float* dists, int nthreads) {
  int64_t qi;
#pragma omp parallel num_threads(nthreads)
  {
    entry* C = (entry*)malloc((size_t)(c_max + 1) * sizeof(entry));
#pragma omp for schedule(dynamic, 4)
    for (qi = 0; qi < (int64_t)nq; ++qi) {
      const char* q = (const char*)queries + (size_t)qi * ix->d * dt_size(ix->dtype);
      uint32_t nc = 0;
      for (uint32_t i = 0; i < c_max; ++i) {
        uint32_t x = cand[qi * c_max + i];
        if (x == OR_NONE || x >= ix->n) continue;
        C[nc].id = x;
        C[nc].dist = 0.0f;
        C[nc].visited = 0;
        ++nc;
      }
      rerank_entries(ix, q, C, nc, nc, k, ids + qi * k, dists + qi * k);
    }
    free(C);
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Precision form of the re-rank, float data only.  The paper re-ranks in
 * FP32 (section "Re-ranking"); this form reads the base rows rounded to
 * bfloat16, sums in FP32, and recomputes in FP32 every candidate that
 * could still be among the k nearest.  Its answer is the FP32 re-rank's by
 * construction: the band E below bounds the gap between the BF16 sum and
 * the canonical FP32 distance of every candidate.
 *
 * Derivation (u = 2^-24, u_b = 2^-8 the unit roundoffs of FP32 and BF16,
 * x~ = bf16(x), D = canonical FP32 distance, D* = exact real distance,
 * D~ = the FP32 sum over x~, D~* its exact value, B = sum of x~^2, and
 * g = (d+2)u/(1-(d+2)u) <= 6.2e-5 for d <= 1024):
 *   |D - D*| <= g D*,  |D~ - D~*| <= g D~*  (sequential sums of squares);
 *   |x~ - x| <= u_b |x| and |x| <= |x~| / (1 - u_b), so with v = u_b/(1-u_b)
 *   |D~* - D*| <= sum |x~ - x| (|x~ - q| + |x - q|)
 *             <= 2v sum |x~||x~ - q| + v^2 B <= 2v sqrt(B D~*) + v^2 B
 *   (Cauchy-Schwarz).  2v = 0.00784 and v^2 = 1.54e-5, so
 *   E = 2^-6 sqrt(B D~) + 2^-15 B + 2^-12 D~
 * bounds |D~ - D| with a factor of two to spare in every term, which also
 * covers the roundings of E, of B and D~ themselves and of D~ -/+ E.
 * ---------------------------------------------------------------------- */

/* x rounded to bfloat16 (8 significant bits, FP32's exponent range) to
 * the nearest, ties to the even significand, returned widened to FP32.
 * The two neighbours in BF16 are x with its low 16 bits cleared and that
 * plus one BF16 step; the nearer wins. */
float or_bf16_round(float x) {
  if (!isfinite(x)) return x;
  uint32_t b;
  memcpy(&b, &x, 4);
  uint32_t lo_b = b & 0xFFFF0000u;          /* toward zero */
  uint32_t hi_b = lo_b + 0x10000u;           /* one step away from zero */
  float lo, hi;
  memcpy(&lo, &lo_b, 4);
  memcpy(&hi, &hi_b, 4);
  double dl = fabs((double)x - (double)lo);
  double dh = fabs((double)hi - (double)x);
  if (dl < dh) return lo;
  if (dh < dl) return hi;
  return ((lo_b >> 16) & 1u) ? hi : lo;      /* tie: the even one */
}

/* D~, B, E and the bounds [lower, upper] of one candidate row x. */
static void bf16_terms(const float* x, const float* q, uint32_t d, float* dt,
                       float* lower, float* upper) {
  float acc = 0.0f, nb = 0.0f;
  for (uint32_t t = 0; t < d; ++t) {
    float xb = or_bf16_round(x[t]);
    float diff = xb - q[t];
    float sq = diff * diff;
    acc = acc + sq;
  }
  for (uint32_t t = 0; t < d; ++t) {
    float xb = or_bf16_round(x[t]);
    float sq = xb * xb;
    nb = nb + sq;
  }
  float bd = nb * acc;
  float e1 = sqrtf(bd) * 0.015625f;          /* 2^-6 */
  float e2 = nb * 3.0517578125e-05f;         /* 2^-15 */
  float e3 = acc * 2.44140625e-04f;          /* 2^-12 */
  float E = (e1 + e2) + e3;
  float lo = acc - E;
  *dt = acc;
  *lower = lo > 0.0f ? lo : 0.0f;
  *upper = acc + E;
}

/* The band of each of n candidates (no padding) of one query, for tests:
 * D~, lower and upper bounds. */
void or_bf16_band(const or_index* ix, const float* q, const uint32_t* ids,
                  uint64_t n, float* dt, float* lower, float* upper) {
  for (uint64_t i = 0; i < n; ++i)
    bf16_terms((const float*)ix->base + (uint64_t)ids[i] * ix->d, q, ix->d,
               dt + i, lower + i, upper + i);
}

typedef struct {
  float key;
  uint32_t id;
} fkey;

static int fkey_cmp(const void* a, const void* b) {
  const fkey* x = (const fkey*)a;
  const fkey* y = (const fkey*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

/* The BF16 re-rank of given candidates (float data): tau = the k-th
 * smallest upper bound (+inf with k or fewer candidates); every candidate
 * whose lower bound is <= tau gets its canonical FP32 distance; the k
 * smallest of those by (distance, id) are the answer.  rechecked[q] = how
 * many were recomputed.  Ids NONE or >= n are padding. */
int or_rerank_bf16(const or_index* ix, const float* queries, uint64_t nq,
                   const uint32_t* cand, uint32_t c_max, uint32_t k,
                   uint32_t* ids, float* dists, uint32_t* rechecked) {
  if (ix->dtype != OR_F32) return -1;
  fkey* U = (fkey*)malloc((size_t)(c_max + 1) * sizeof(fkey));
  float* lo = (float*)malloc((size_t)(c_max + 1) * sizeof(float));
  uint32_t* id = (uint32_t*)malloc((size_t)(c_max + 1) * sizeof(uint32_t));
  entry* C = (entry*)malloc((size_t)(c_max + 1) * sizeof(entry));
  if (!U || !lo || !id || !C) {
    free(U); free(lo); free(id); free(C);
    return -2;
  }
  for (uint64_t qi = 0; qi < nq; ++qi) {
    const float* q = queries + qi * ix->d;
    uint32_t nc = 0;
    for (uint32_t i = 0; i < c_max; ++i) {
      uint32_t x = cand[qi * c_max + i];
      if (x == OR_NONE || x >= ix->n) continue;
      float dt, up;
      bf16_terms((const float*)ix->base + (uint64_t)x * ix->d, q, ix->d, &dt,
                 &lo[nc], &up);
      U[nc].key = up;
      U[nc].id = x;
      id[nc] = x;
      ++nc;
    }
    float tau = INFINITY;
    if (nc > k) {
      fkey* S = (fkey*)malloc((size_t)nc * sizeof(fkey));
      memcpy(S, U, (size_t)nc * sizeof(fkey));
      qsort(S, nc, sizeof(fkey), fkey_cmp);
      tau = S[k - 1].key;
      free(S);
    }
    uint32_t nr = 0;
    for (uint32_t i = 0; i < nc; ++i) {
      if (!(lo[i] <= tau)) continue;
      C[nr].id = id[i];
      C[nr].dist = exact_dist(ix, q, id[i]);
      C[nr].visited = 0;
      ++nr;
    }
    qsort(C, nr, sizeof(entry), entry_cmp);
    for (uint32_t i = 0; i < k; ++i) {
      ids[qi * k + i] = i < nr ? C[i].id : OR_NONE;
      dists[qi * k + i] = i < nr ? C[i].dist : INFINITY;
    }
    if (rechecked) rechecked[qi] = nr;
  }
  free(U);
  free(lo);
  free(id);
  free(C);
  return 0;
}

/* ------------------------------------------------------------------------
 * Ground truth: brute-force exact k nearest (the kNN problem statement in
 * the introduction; recall definition in "Algorithm Parameters").  Integer
 * data is exact in int64; float data in FP64.  Ordered by (dist, id).
 * Queries are processed in blocks of QB so each base row is read once per
 * block; the result does not depend on the block size.
 * ---------------------------------------------------------------------- */
#define QB 16
static void topk_insert(double* bd, uint32_t* bi, uint32_t k, double dv,
                        uint32_t id) {
  /* keep (bd, bi) sorted by (dist, id); insert if better than the last */
  if (dv > bd[k - 1] || (dv == bd[k - 1] && id >= bi[k - 1])) return;
  int64_t p = (int64_t)k - 1;
  while (p > 0 && (bd[p - 1] > dv || (bd[p - 1] == dv && bi[p - 1] > id))) {
    bd[p] = bd[p - 1];
    bi[p] = bi[p - 1];
    --p;
  }
  bd[p] = dv;
  bi[p] = id;
}

int or_bruteforce(const void* base, int dt, uint64_t n, uint32_t d,
                  const void* queries, uint64_t nq, uint32_t k, uint32_t* ids,
                  double* dists, int nthreads) {
  if (k == 0) return -1;
  int64_t blk;
  int64_t nblk = (int64_t)((nq + QB - 1) / QB);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (blk = 0; blk < nblk; ++blk) {
    uint64_t q0 = (uint64_t)blk * QB;
    uint64_t q1 = q0 + QB < nq ? q0 + QB : nq;
    double bd[QB][256 + 1];
    uint32_t bi[QB][256 + 1];
    double* bdp[QB];
    uint32_t* bip[QB];
    double* heapd = NULL;
    uint32_t* heapi = NULL;
    if (k > 256) {
      heapd = (double*)malloc(sizeof(double) * QB * k);
      heapi = (uint32_t*)malloc(sizeof(uint32_t) * QB * k);
    }
    for (uint64_t a = 0; a < q1 - q0; ++a) {
      bdp[a] = heapd ? heapd + a * k : bd[a];
      bip[a] = heapi ? heapi + a * k : bi[a];
      for (uint32_t i = 0; i < k; ++i) {
        bdp[a][i] = INFINITY;
        bip[a][i] = OR_NONE;
      }
    }
    for (uint64_t x = 0; x < n; ++x) {
      for (uint64_t a = 0; a < q1 - q0; ++a) {
        uint64_t qq = q0 + a;
        double dv;
        if (dt == OR_F32) {
          const float* xr = (const float*)base + x * d;
          const float* qr = (const float*)queries + qq * d;
          double acc = 0.0;
          for (uint32_t t = 0; t < d; ++t) {
            double diff = (double)xr[t] - (double)qr[t];
            acc += diff * diff;
          }
          dv = acc;
        } else if (dt == OR_U8) {
          const uint8_t* xr = (const uint8_t*)base + x * d;
          const uint8_t* qr = (const uint8_t*)queries + qq * d;
          int32_t acc = 0;
          for (uint32_t t = 0; t < d; ++t) {
            int32_t diff = (int32_t)xr[t] - (int32_t)qr[t];
            acc += diff * diff;
          }
          dv = (double)acc;
        } else {
          const int8_t* xr = (const int8_t*)base + x * d;
          const int8_t* qr = (const int8_t*)queries + qq * d;
          int32_t acc = 0;
          for (uint32_t t = 0; t < d; ++t) {
            int32_t diff = (int32_t)xr[t] - (int32_t)qr[t];
            acc += diff * diff;
          }
          dv = (double)acc;
        }
        topk_insert(bdp[a], bip[a], k, dv, (uint32_t)x);
      }
    }
    for (uint64_t a = 0; a < q1 - q0; ++a)
      for (uint32_t i = 0; i < k; ++i) {
        ids[(q0 + a) * k + i] = bip[a][i];
        dists[(q0 + a) * k + i] = bdp[a][i];
      }
    free(heapd);
    free(heapi);
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * PQ (section "Construction of PQDistTable" describes the compression: the
 * d dimensions split into m contiguous subspaces, 256 k-means centroids per
 * subspace, each vector stored as m one-byte centroid ids).
 * ---------------------------------------------------------------------- */

/* Lloyd assignment step: nearest centroid in FP64, ties to the lowest id.
 * X[n][ds] and Cen[K][ds] are FP64.  Returns the objective. */
double or_kmeans_assign(const double* X, uint64_t n, uint32_t ds,
                        const double* Cen, uint32_t K, int32_t* assign,
                        int nthreads) {
  double obj = 0.0;
  int64_t i;
#pragma omp parallel for schedule(static) reduction(+ : obj) num_threads(nthreads)
  for (i = 0; i < (int64_t)n; ++i) {
    double best = INFINITY;
    int32_t bc = 0;
    for (uint32_t c = 0; c < K; ++c) {
      double acc = 0.0;
      for (uint32_t t = 0; t < ds; ++t) {
        double diff = X[(uint64_t)i * ds + t] - Cen[(uint64_t)c * ds + t];
        acc += diff * diff;
      }
      if (acc < best) {
        best = acc;
        bc = (int32_t)c;
      }
    }
    assign[i] = bc;
    obj += best;
  }
  return obj;
}

/* Encoding: code[i][j] = arg min_c ||x_i^(j) - cb[j][c]||^2 in FP64, ties to
 * the lowest c.  X is in its own element type. */
void or_pq_encode(const void* X, int dt, uint64_t n, uint32_t d,
                  const float* cb, uint32_t m, uint8_t* codes, int nthreads) {
  uint32_t ds = d / m;
  int64_t i;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (i = 0; i < (int64_t)n; ++i) {
    for (uint32_t j = 0; j < m; ++j) {
      double best = INFINITY;
      uint32_t bc = 0;
      for (uint32_t c = 0; c < 256; ++c) {
        double acc = 0.0;
        for (uint32_t t = 0; t < ds; ++t) {
          double diff = elem_d(X, dt, (uint64_t)i * d + (uint64_t)j * ds + t) -
                        (double)cb[((uint64_t)j * 256 + c) * ds + t];
          acc += diff * diff;
        }
        if (acc < best) {
          best = acc;
          bc = c;
        }
      }
      codes[(uint64_t)i * m + j] = (uint8_t)bc;
    }
  }
}

/* ------------------------------------------------------------------------
 * Vamana graph (named in "Graph Index" and "Algorithm Parameters"; built
 * offline with DiskANN in the paper, which gives R, L and alpha but not the
 * procedure).  This follows the published Vamana method: greedy search from
 * the medoid to collect the visited set, RobustPrune with parameter alpha
 * to choose at most R out-neighbours, then back-edges that re-prune any
 * list that grows past its capacity.  Insertions run in batches whose size
 * doubles from 1 up to max_batch; inside a batch every search reads the
 * graph as it was at the batch start, so the result does not depend on the
 * thread count.
 * ---------------------------------------------------------------------- */
typedef struct {
  const void* base;
  int dt;
  uint64_t n;
  uint32_t d;
} vset;

static double vdist(const vset* v, uint32_t a, uint32_t b) {
  uint32_t d = v->d;
  if (v->dt == OR_U8) {
    const uint8_t* x = (const uint8_t*)v->base + (uint64_t)a * d;
    const uint8_t* y = (const uint8_t*)v->base + (uint64_t)b * d;
    int32_t acc = 0;
    for (uint32_t t = 0; t < d; ++t) {
      int32_t df = (int32_t)x[t] - (int32_t)y[t];
      acc += df * df;
    }
    return (double)acc;
  }
  if (v->dt == OR_I8) {
    const int8_t* x = (const int8_t*)v->base + (uint64_t)a * d;
    const int8_t* y = (const int8_t*)v->base + (uint64_t)b * d;
    int32_t acc = 0;
    for (uint32_t t = 0; t < d; ++t) {
      int32_t df = (int32_t)x[t] - (int32_t)y[t];
      acc += df * df;
    }
    return (double)acc;
  }
  const float* x = (const float*)v->base + (uint64_t)a * d;
  const float* y = (const float*)v->base + (uint64_t)b * d;
  double acc = 0.0;
  for (uint32_t t = 0; t < d; ++t) {
    double df = (double)x[t] - (double)y[t];
    acc += df * df;
  }
  return acc;
}

typedef struct {
  double dist;
  uint32_t id;
  int32_t flag;
} dentry;

static int dentry_cmp(const void* a, const void* b) {
  const dentry* x = (const dentry*)a;
  const dentry* y = (const dentry*)b;
  if (x->dist < y->dist) return -1;
  if (x->dist > y->dist) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* Medoid: the point closest to the mean of all points (FP64), ties to the
 * lowest id. */
uint32_t or_medoid(const void* base, int dt, uint64_t n, uint32_t d) {
  double* mean = (double*)calloc(d, sizeof(double));
  for (uint64_t i = 0; i < n; ++i)
    for (uint32_t t = 0; t < d; ++t) mean[t] += elem_d(base, dt, i * d + t);
  for (uint32_t t = 0; t < d; ++t) mean[t] /= (double)n;
  double best = INFINITY;
  uint32_t bi = 0;
  for (uint64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (uint32_t t = 0; t < d; ++t) {
      double df = elem_d(base, dt, i * d + t) - mean[t];
      acc += df * df;
    }
    if (acc < best) {
      best = acc;
      bi = (uint32_t)i;
    }
  }
  free(mean);
  return bi;
}

typedef struct {
  uint32_t* nbr; /* n * cap */
  uint32_t* deg; /* n */
  uint32_t cap;
} vgraph;

/* Greedy search toward point p with a worklist of Lb entries; returns the
 * expanded (visited) nodes in V. */
static uint32_t vgreedy(const vset* v, const vgraph* g, uint32_t s, uint32_t p,
                        uint32_t Lb, uint32_t* seen, uint32_t stamp, dentry* L,
                        dentry* tmp, uint32_t* V, uint32_t vcap) {
  uint32_t len = 1, nv = 0;
  L[0].dist = vdist(v, s, p);
  L[0].id = s;
  L[0].flag = 0;
  seen[s] = stamp;
  for (;;) {
    int64_t pos = -1;
    for (uint32_t i = 0; i < len; ++i)
      if (!L[i].flag) {
        pos = i;
        break;
      }
    if (pos < 0 || nv == vcap) break;
    L[pos].flag = 1;
    uint32_t u = L[pos].id;
    V[nv++] = u;
    uint32_t nn = 0;
    for (uint32_t r = 0; r < g->deg[u]; ++r) {
      uint32_t x = g->nbr[(uint64_t)u * g->cap + r];
      if (seen[x] == stamp) continue;
      seen[x] = stamp;
      tmp[nn].dist = vdist(v, x, p);
      tmp[nn].id = x;
      tmp[nn].flag = 0;
      ++nn;
    }
    qsort(tmp, nn, sizeof(dentry), dentry_cmp);
    /* merge tmp into L keeping Lb */
    dentry* out = tmp + g->cap;
    uint32_t a = 0, b = 0, o = 0;
    while (o < Lb && (a < len || b < nn)) {
      if (b >= nn || (a < len && dentry_cmp(&L[a], &tmp[b]) < 0))
        out[o++] = L[a++];
      else
        out[o++] = tmp[b++];
    }
    memcpy(L, out, o * sizeof(dentry));
    len = o;
  }
  return nv;
}

/* RobustPrune(p, cand, alpha, R): candidates in (distance to p, id) order;
 * take the nearest, drop every remaining p' with
 * alpha * d(p*, p') <= d(p, p') (non-squared distances, i.e.
 * alpha^2 * d2(p*, p') <= d2(p, p')), repeat until R are chosen. */
static uint32_t robust_prune(const vset* v, uint32_t p, const uint32_t* cand,
                             uint32_t nc, double alpha, uint32_t R,
                             dentry* work, uint32_t* out) {
  uint32_t w = 0;
  for (uint32_t i = 0; i < nc; ++i) {
    uint32_t x = cand[i];
    if (x == p) continue;
    work[w].dist = vdist(v, p, x);
    work[w].id = x;
    work[w].flag = 1; /* alive */
    ++w;
  }
  qsort(work, w, sizeof(dentry), dentry_cmp);
  /* a repeated candidate sorts next to its first copy: drop the repeats */
  uint32_t u = 0;
  for (uint32_t i = 0; i < w; ++i)
    if (u == 0 || work[i].id != work[u - 1].id) work[u++] = work[i];
  w = u;
  double a2 = alpha * alpha;
  uint32_t no = 0;
  for (uint32_t i = 0; i < w && no < R; ++i) {
    if (!work[i].flag) continue;
    out[no++] = work[i].id;
    work[i].flag = 0;
    for (uint32_t j = i + 1; j < w; ++j) {
      if (!work[j].flag) continue;
      if (a2 * vdist(v, work[i].id, work[j].id) <= work[j].dist) work[j].flag = 0;
    }
  }
  return no;
}

/* RobustPrune alone, for the tests: the at most R out-neighbours of point
 * p chosen from cand[0..nc) (repeats and p itself allowed in cand), in
 * selection order.  Returns their count, or -2 when out of memory. */
int64_t or_robust_prune(const void* base, int dt, uint64_t n, uint32_t d,
                        uint32_t p, const uint32_t* cand, uint32_t nc,
                        double alpha, uint32_t R, uint32_t* out) {
  vset v = {base, dt, n, d};
  dentry* work = (dentry*)malloc(sizeof(dentry) * (nc ? nc : 1));
  if (!work) return -2;
  uint32_t no = robust_prune(&v, p, cand, nc, alpha, R, work, out);
  free(work);
  return (int64_t)no;
}

typedef struct {
  uint32_t tgt;
  uint32_t src;
} edge;

static int edge_cmp(const void* a, const void* b) {
  const edge* x = (const edge*)a;
  const edge* y = (const edge*)b;
  if (x->tgt != y->tgt) return (x->tgt > y->tgt) - (x->tgt < y->tgt);
  return (x->src > y->src) - (x->src < y->src);
}

/*
 * Build.  perm: insertion order (length n); alphas[npass]: one pass each;
 * slack: a list may grow to floor(slack*R) entries through back-edges
 * before it is pruned back to R; a final sweep prunes every list still
 * longer than R with the last alpha.  adj_out[n][R] gets OR_NONE padding.
 */
int or_vamana_build(const void* base, int dt, uint64_t n, uint32_t d,
                    uint32_t R, uint32_t Lb, const double* alphas, int npass,
                    const uint32_t* perm, uint32_t medoid, double slack,
                    uint32_t max_batch, uint32_t* adj_out, int nthreads) {
  vset v = {base, dt, n, d};
  vgraph g;
  uint32_t cap = (uint32_t)floor(slack * R);
  if (cap < R) cap = R;
  g.cap = cap;
  g.nbr = (uint32_t*)malloc(sizeof(uint32_t) * n * cap);
  g.deg = (uint32_t*)calloc(n, sizeof(uint32_t));
  uint32_t* newn = (uint32_t*)malloc(sizeof(uint32_t) * (uint64_t)max_batch * R);
  uint32_t* newdeg = (uint32_t*)malloc(sizeof(uint32_t) * max_batch);
  edge* edges = (edge*)malloc(sizeof(edge) * (uint64_t)max_batch * R);
  uint64_t* gstart = (uint64_t*)malloc(sizeof(uint64_t) * ((uint64_t)max_batch * R + 1));
  if (!g.nbr || !g.deg || !newn || !newdeg || !edges || !gstart) return -2;
  uint32_t vcap = 4 * Lb + 64;
  for (int pass = 0; pass < npass; ++pass) {
    double alpha = alphas[pass];
    uint64_t start = 0, bsz = 1;
    while (start < n) {
      uint64_t end = start + bsz < n ? start + bsz : n;
      int64_t i;
      /* 1) search + prune for every point of the batch (graph frozen) */
#pragma omp parallel num_threads(nthreads)
      {
        uint32_t* seen = (uint32_t*)calloc(n, sizeof(uint32_t));
        uint32_t stamp = 0;
        dentry* L = (dentry*)malloc(sizeof(dentry) * (Lb + cap));
        dentry* tmp = (dentry*)malloc(sizeof(dentry) * (2 * cap + Lb));
        uint32_t* V = (uint32_t*)malloc(sizeof(uint32_t) * (vcap + cap));
        dentry* work = (dentry*)malloc(sizeof(dentry) * (vcap + cap));
#pragma omp for schedule(dynamic, 1)
        for (i = (int64_t)start; i < (int64_t)end; ++i) {
          uint32_t p = perm[i];
          ++stamp;
          uint32_t nv = vgreedy(&v, &g, medoid, p, Lb, seen, stamp, L, tmp, V, vcap);
          for (uint32_t r = 0; r < g.deg[p]; ++r) V[nv++] = g.nbr[(uint64_t)p * cap + r];
          newdeg[i - start] = robust_prune(&v, p, V, nv, alpha, R, work,
                                           newn + (uint64_t)(i - start) * R);
        }
        free(seen);
        free(L);
        free(tmp);
        free(V);
        free(work);
      }
      /* 2) install the new lists */
      uint64_t ne = 0;
      for (uint64_t b = start; b < end; ++b) {
        uint32_t p = perm[b];
        uint32_t dg = newdeg[b - start];
        memcpy(g.nbr + (uint64_t)p * cap, newn + (b - start) * R, dg * sizeof(uint32_t));
        g.deg[p] = dg;
        for (uint32_t r = 0; r < dg; ++r) {
          edges[ne].tgt = g.nbr[(uint64_t)p * cap + r];
          edges[ne].src = p;
          ++ne;
        }
      }
      /* 3) back-edges, grouped by target */
      qsort(edges, ne, sizeof(edge), edge_cmp);
      uint64_t ng = 0;
      for (uint64_t e = 0; e < ne; ++e)
        if (e == 0 || edges[e].tgt != edges[e - 1].tgt) gstart[ng++] = e;
      gstart[ng] = ne;
#pragma omp parallel num_threads(nthreads)
      {
        uint32_t* cand = (uint32_t*)malloc(sizeof(uint32_t) * (cap + max_batch));
        dentry* work = (dentry*)malloc(sizeof(dentry) * (cap + max_batch));
        uint32_t* out = (uint32_t*)malloc(sizeof(uint32_t) * R);
#pragma omp for schedule(dynamic, 16)
        for (i = 0; i < (int64_t)ng; ++i) {
          uint32_t j = edges[gstart[i]].tgt;
          uint32_t nc = g.deg[j];
          memcpy(cand, g.nbr + (uint64_t)j * cap, nc * sizeof(uint32_t));
          for (uint64_t e = gstart[i]; e < gstart[i + 1]; ++e) {
            uint32_t src = edges[e].src;
            int present = (src == j);
            for (uint32_t r = 0; r < nc && !present; ++r)
              if (cand[r] == src) present = 1;
            if (!present) cand[nc++] = src;
          }
          if (nc <= cap) {
            memcpy(g.nbr + (uint64_t)j * cap, cand, nc * sizeof(uint32_t));
            g.deg[j] = nc;
          } else {
            uint32_t no = robust_prune(&v, j, cand, nc, alpha, R, work, out);
            memcpy(g.nbr + (uint64_t)j * cap, out, no * sizeof(uint32_t));
            g.deg[j] = no;
          }
        }
        free(cand);
        free(work);
        free(out);
      }
      start = end;
      bsz = bsz * 2 < max_batch ? bsz * 2 : max_batch;
    }
  }
  /* final sweep: every list longer than R is pruned back to R */
  {
    double alpha = alphas[npass - 1];
    int64_t j;
#pragma omp parallel num_threads(nthreads)
    {
      dentry* work = (dentry*)malloc(sizeof(dentry) * cap);
      uint32_t* out = (uint32_t*)malloc(sizeof(uint32_t) * R);
      uint32_t* cand = (uint32_t*)malloc(sizeof(uint32_t) * cap);
#pragma omp for schedule(dynamic, 64)
      for (j = 0; j < (int64_t)n; ++j) {
        if (g.deg[j] <= R) continue;
        memcpy(cand, g.nbr + (uint64_t)j * cap, g.deg[j] * sizeof(uint32_t));
        uint32_t no = robust_prune(&v, (uint32_t)j, cand, g.deg[j], alpha, R, work, out);
        memcpy(g.nbr + (uint64_t)j * cap, out, no * sizeof(uint32_t));
        g.deg[j] = no;
      }
      free(work);
      free(out);
      free(cand);
    }
  }
  for (uint64_t j = 0; j < n; ++j)
    for (uint32_t r = 0; r < R; ++r)
      adj_out[j * R + r] = r < g.deg[j] ? g.nbr[j * cap + r] : OR_NONE;
  free(g.nbr);
  free(g.deg);
  free(newn);
  free(newdeg);
  free(edges);
  free(gstart);
  return 0;
}

/* Nodes reachable from s (breadth-first). */
uint64_t or_reachable(const uint32_t* adj, uint64_t n, uint32_t R, uint32_t s) {
  uint8_t* mark = (uint8_t*)calloc(n, 1);
  uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint64_t head = 0, tail = 0;
  mark[s] = 1;
  queue[tail++] = s;
  while (head < tail) {
    uint32_t u = queue[head++];
    for (uint32_t r = 0; r < R; ++r) {
      uint32_t x = adj[(uint64_t)u * R + r];
      if (x == OR_NONE || x >= n || mark[x]) continue;
      mark[x] = 1;
      queue[tail++] = x;
    }
  }
  free(mark);
  free(queue);
  return tail;
}

int or_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------
 * Connectivity repair (a reading: the paper's graphs come from DiskANN and
 * it does not discuss unreachable nodes; search from one start node needs
 * every node reachable from it).  Following the NSG method: for each node
 * not reachable from s, in increasing id order, run the build's greedy
 * search from s toward it, and add an edge from the nearest visited node
 * that still has a free slot (else the nearest visited node, replacing its
 * last neighbour).  Reachability is then extended from the new node.  The
 * sweep repeats until every node is reachable or max_rounds is reached.
 * Returns the number of edges added.
 * ---------------------------------------------------------------------- */
static void mark_from(const uint32_t* adj, uint64_t n, uint32_t R, uint32_t s,
                      uint8_t* mark, uint32_t* queue) {
  uint64_t head = 0, tail = 0;
  if (mark[s]) return;
  mark[s] = 1;
  queue[tail++] = s;
  while (head < tail) {
    uint32_t u = queue[head++];
    for (uint32_t r = 0; r < R; ++r) {
      uint32_t x = adj[(uint64_t)u * R + r];
      if (x == OR_NONE || x >= n || mark[x]) continue;
      mark[x] = 1;
      queue[tail++] = x;
    }
  }
}

int64_t or_connect(const void* base, int dt, uint64_t n, uint32_t d,
                   uint32_t* adj, uint32_t R, uint32_t s, uint32_t Lb,
                   int max_rounds) {
  vset v = {base, dt, n, d};
  vgraph g;
  g.cap = R;
  g.nbr = adj;
  g.deg = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint8_t* mark = (uint8_t*)malloc(n);
  uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint32_t* seen = (uint32_t*)calloc(n, sizeof(uint32_t));
  uint32_t vcap = 4 * Lb + 64;
  dentry* L = (dentry*)malloc(sizeof(dentry) * (Lb + R));
  dentry* tmp = (dentry*)malloc(sizeof(dentry) * (2 * R + Lb));
  uint32_t* V = (uint32_t*)malloc(sizeof(uint32_t) * vcap);
  dentry* order = (dentry*)malloc(sizeof(dentry) * vcap);
  uint32_t* indeg = (uint32_t*)malloc(sizeof(uint32_t) * n);
  int64_t added = 0;
  uint32_t stamp = 0;
  for (int round = 0; round < max_rounds; ++round) {
    /* compact every row: its valid ids first, in stored order */
    for (uint64_t j = 0; j < n; ++j) {
      uint32_t c = 0;
      for (uint32_t r = 0; r < R; ++r) {
        uint32_t x = adj[j * R + r];
        if (x != OR_NONE) adj[j * R + c++] = x;
      }
      for (uint32_t r = c; r < R; ++r) adj[j * R + r] = OR_NONE;
      g.deg[j] = c;
    }
    memset(indeg, 0, sizeof(uint32_t) * n);
    for (uint64_t j = 0; j < n * R; ++j)
      if (adj[j] != OR_NONE) indeg[adj[j]]++;
    memset(mark, 0, n);
    mark_from(adj, n, R, s, mark, queue);
    int64_t before = added;
    for (uint64_t u = 0; u < n; ++u) {
      if (mark[u]) continue;
      ++stamp;
      uint32_t nv = vgreedy(&v, &g, s, (uint32_t)u, Lb, seen, stamp, L, tmp, V, vcap);
      for (uint32_t i = 0; i < nv; ++i) {
        order[i].dist = vdist(&v, V[i], (uint32_t)u);
        order[i].id = V[i];
        order[i].flag = 0;
      }
      qsort(order, nv, sizeof(dentry), dentry_cmp);
      /* nearest visited node with a free slot; failing that, the nearest
       * one whose last neighbour keeps another in-edge after the swap */
      uint32_t pick = order[0].id;
      int freeslot = 0;
      for (uint32_t i = 0; i < nv; ++i)
        if (g.deg[order[i].id] < R) {
          pick = order[i].id;
          freeslot = 1;
          break;
        }
      if (!freeslot)
        for (uint32_t i = 0; i < nv; ++i)
          if (indeg[adj[(uint64_t)order[i].id * R + R - 1]] >= 2) {
            pick = order[i].id;
            break;
          }
      if (freeslot) {
        adj[(uint64_t)pick * R + g.deg[pick]] = (uint32_t)u;
        g.deg[pick]++;
      } else {
        indeg[adj[(uint64_t)pick * R + R - 1]]--;
        adj[(uint64_t)pick * R + R - 1] = (uint32_t)u;
      }
      indeg[u]++;
      ++added;
      mark_from(adj, n, R, (uint32_t)u, mark, queue);
    }
    if (added == before) break;
  }
  free(g.deg);
  free(indeg);
  free(mark);
  free(queue);
  free(seen);
  free(L);
  free(tmp);
  free(V);
  free(order);
  return added;
}
