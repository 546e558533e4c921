/*
 * bang.h: C ABI of the MI355X (gfx950) batched PQ graph search.
 *
 * The library implements the three GPU stages of BANG (arXiv 2401.11324,
 * section "BANG: Billion-scale ANNS on a Single GPU"): (1) the PQ distance
 * table, (2) the greedy search over a proximity graph with asymmetric (PQ)
 * distances (Algorithms 1 and 2), and (3) the exact re-rank.  The graph and
 * the compressed vectors live in device memory, as in the paper's
 * "In-memory Version" (section "Implementation Variants"), or the adjacency
 * stays in pinned host memory (BANG_INDEX_HOST_ADJ), as in the base design.
 * Options select the table storage (FP32, the FP16 / u8 precision forms,
 * or the paper's Exact-distance Version), the visited filter (set union or
 * the paper's Bloom filter) and mixed per-query k and L; a serving loop
 * (bang_server_*) batches requests continuously, and bang_index_probe
 * measures the rate at which the search's rows can be read.
 *
 * Conventions shared by every call:
 *  - Status: every call returns 0 on success or a negative BANG_E* code;
 *    bang_last_error() then describes the failure (thread-local string).
 *    Validation happens on the host before any launch: a call that fails
 *    validation launches nothing and writes nothing.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls are asynchronous and stream-ordered; outputs are valid
 *    once the caller synchronises the stream.
 *  - Ownership: the caller owns every query and output buffer (device
 *    pointers, e.g. from torch tensors).  The index owns its device copies
 *    of the base vectors, adjacency, codebooks and codes, and a workspace
 *    reused by every search on it: searches on one index must not overlap
 *    in time (use one index per concurrent stream).
 *  - Distances are squared Euclidean (the paper builds its table from
 *    squared distances).  Results are ordered by (distance, id).
 *  - Arithmetic: FP32 with no fused multiply-add, summed in a fixed order:
 *    table entry = sum over the d/m coordinates, ADC = sum over the m
 *    subspaces in index order, exact distance of float data = sum over the
 *    d coordinates in order; integer data (u8/i8) uses an exact integer
 *    sum converted once to FP32.
 */
#ifndef BANG_H_
#define BANG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BANG_OK 0
#define BANG_EINVAL (-1)       /* invalid argument */
#define BANG_ENOMEM (-2)       /* allocation failed / over the memory budget */
#define BANG_EDEVICE (-3)      /* HIP runtime error or no usable GPU */
#define BANG_EUNSUPPORTED (-4) /* valid but not supported by this build */
#define BANG_EABORTED (-5)     /* stopped by a stop request, or a wait
                                  that timed out */

#define BANG_NONE 0xFFFFFFFFu  /* empty adjacency slot / padded result id */
#define BANG_MAX_L 1024u       /* largest worklist (the paper's t) */
#define BANG_MAX_R 64u         /* largest graph degree */

typedef enum { BANG_F32 = 0, BANG_U8 = 1, BANG_I8 = 2 } bang_dtype;

typedef struct bang_index bang_index; /* opaque */
typedef struct bang_abort bang_abort; /* opaque: a stop request */

/* Index description; every pointer is HOST memory, read during
 * bang_index_create only. */
typedef struct {
  uint64_t n;               /* number of base vectors, 1 <= n < 2^31 */
  uint32_t d;               /* dimension */
  int32_t dtype;            /* bang_dtype of base vectors and queries */
  const void* base;         /* [n][d] row-major */
  uint32_t R;               /* graph degree bound, 1..BANG_MAX_R */
  const uint32_t* adj;      /* [n][R]; ids < n or BANG_NONE; no id twice
                               in a row */
  uint32_t medoid;          /* start node s (Algorithm 1), < n */
  uint32_t m;               /* PQ subspaces; m divides d */
  const float* codebooks;   /* [m][256][d/m] FP32 centroids */
  const uint8_t* codes;     /* [n][m] centroid ids */
  uint32_t flags;           /* 0, BANG_INDEX_HOST_ADJ, BANG_INDEX_BF16_BASE */
} bang_index_desc;

/* Index flag: keep the adjacency in pinned host memory instead of device
 * memory, the paper's CPU-resident graph (section "BANG: Billion-scale ANNS
 * on a Single GPU": the graph stays in host RAM, the compressed vectors on
 * the GPU).  bang_index_create copies adj into a page-locked host buffer
 * (hipHostMalloc, GPU-cacheable, read-only after create); the search
 * kernel reads one adjacency row (4R bytes) across the host link per
 * expansion and gathers the neighbours' codes from device memory.  Base
 * vectors, codes and codebooks stay in device memory.  Results are the
 * same as with a device-resident graph. */
#define BANG_INDEX_HOST_ADJ 1u

/* Index flag, float data with d a multiple of 8: also keep the base rounded
 * to bfloat16 (nearest, ties to even; 2 bytes a coordinate) and the sum of
 * squares of each rounded row (FP32, coordinates in order), for the
 * precision form's re-rank (bang_search_opts.rerank = BANG_RERANK_BF16).
 * Device memory: n*d*2 + n*4 bytes more. */
#define BANG_INDEX_BF16_BASE 2u

/* Optional search outputs for inspection; NULL pointers are skipped. */
typedef struct {
  uint32_t c_max;           /* re-rank candidates kept (0 = 4*L): when more
                               nodes were expanded, the c_max smallest by
                               (PQ distance, id) are re-ranked */
  uint32_t iter_cap;        /* iterations per query (0 = max(4L, L + 64)); a
                               query that hits it stops and reports status 1 */
  uint32_t* out_cand;       /* device [nq][cand_stride]: expanded node ids in
                               expansion order, BANG_NONE padded */
  uint32_t cand_stride;
  uint32_t* out_counters;   /* device [nq][4]: {iterations, status,
                               rechecked, 0}; status 0 converged, 1 stopped
                               at iter_cap, 2 stopped by the stop request
                               (abort); rechecked: with BANG_RERANK_BF16 the
                               candidates given an FP32 distance, else 0 */
  uint64_t* out_times;      /* device [nq][2]: device wall-clock ticks when
                               the query's work began and when its results
                               were written (hipDeviceAttributeWallClockRate
                               gives the tick rate in kHz) */
  uint32_t table;           /* storage of the PQ table the search ranks by:
                               BANG_TABLE_F32 (default), the precision
                               form's BANG_TABLE_F16 / BANG_TABLE_U8, or
                               BANG_TABLE_EXACT (no table) */
  uint32_t flags;           /* 0, or BANG_SEARCH_RERANK_GLOBAL |
                               BANG_SEARCH_SEEN_LOG_SHORT |
                               BANG_SEARCH_NO_SEEN_CACHE */
  const uint32_t* query_L;  /* device [nq] or NULL: a mixed batch, query i
                               searched with worklist size L_i in [1, L]
                               and, with query_k, k_i results in
                               [1, min(k, L_i)] (values out of range are
                               clamped); its iteration cap and c_max are
                               the defaults for L_i, so c_max and iter_cap
                               above must be 0.  Row i of the outputs holds
                               k_i results, then (BANG_NONE, +inf) up to k.
                               Each query's result equals a search of that
                               query alone with (k_i, L_i). */
  const uint32_t* query_k;  /* device [nq] or NULL (every k_i = k) */
  uint32_t filter;          /* visited filter: BANG_FILTER_EXACT (default),
                               BANG_FILTER_BLOOM or BANG_FILTER_SEEN */
  uint32_t* out_phases;     /* device [nq][7] or NULL: shader-clock cycles
                               (s_memtime) of each query's phases: table and
                               worklist start; then summed over expansions:
                               waiting for the row, scoring the neighbours,
                               ranking them in the worklist, choosing the
                               next node and requesting its row, merging;
                               then the re-rank.  Runs a timed copy of the
                               search (same results, somewhat slower);
                               device-resident adjacency and no Bloom
                               filter (EUNSUPPORTED otherwise). */
  const bang_abort* abort;  /* NULL, or a stop request (bang_abort_create)
                               this search obeys: once it is set, each wave
                               finishes the expansion it is in, writes its
                               query's row as padding (BANG_NONE, +inf) with
                               status 2 in out_counters, and every query not
                               yet started is written the same way without
                               being searched.  Queries that finished before
                               keep their results. */
  uint32_t rerank;          /* BANG_RERANK_EXACT (default) or
                               BANG_RERANK_BF16 */
  const float* tables;      /* NULL, or device [nq][m][256] FP32 PQ tables
                               built beforehand (bang_build_pq_tables or
                               bang_build_pq_tables_bf16): query i is
                               searched by tables[i] (stored in the table
                               form above) instead of a table the search
                               builds; 4-byte aligned; not with
                               BANG_TABLE_EXACT.  With the tables of
                               bang_build_pq_tables the results are those of
                               the search without this option. */
  const uint32_t* order;    /* NULL, or device [nq]: the order in which the
                               persistent waves take the queries (the t-th
                               query taken is order[t]; a permutation of
                               0..nq-1; an entry >= nq takes query nq-1,
                               which is then searched twice with the same
                               result).  Results
                               stay in each query's own row and do not
                               depend on the order; it sets how the
                               launch's tail is balanced (e.g. the longest
                               worklists first in a mixed batch). */
  uint32_t waves_per_cu;    /* 0, or a cap on the resident waves per CU
                               (at most what LDS and registers allow) */
} bang_search_opts;

/* Re-rank forms (float data; integer data is always re-ranked exactly).
 *  - EXACT: the canonical FP32 distance of every candidate.
 *  - BF16: the precision form's re-rank, same answer.  Each candidate's
 *    distance D~ is first summed in FP32 from its bfloat16 row (half the
 *    bytes); with B its row's sum of squares, E = 2^-6 sqrt(B D~) +
 *    2^-15 B + 2^-12 D~ bounds the gap to its canonical FP32 distance
 *    (d <= 1024).  Every candidate whose D~ - E is at most the k-th
 *    smallest D~ + E, the only ones that can be among the k nearest, is
 *    recomputed in FP32 from the float row, and the k nearest of those by
 *    (FP32 distance, id) are returned: ids and distances equal EXACT's.
 *    Needs an index created with BANG_INDEX_BF16_BASE and a PQ table form.
 *    The re-rank falls back to EXACT when its arrays do not fit on chip
 *    (about 8 bytes per candidate more than EXACT). */
#define BANG_RERANK_EXACT 0u
#define BANG_RERANK_BF16 1u

/* Visited filters.
 *  - EXACT: set union into the worklist (Algorithm 1): a neighbour already
 *    in the worklist is dropped; one evicted from a full worklist can never
 *    re-enter, so this is an exact seen-set.  No extra memory.
 *  - BLOOM: the paper's filter (section "Parallel Filtering of Visited
 *    Neighbours"): per query z = BANG_BLOOM_Z entries and two FNV-1a-32
 *    hashes of the id's four little-endian bytes (offset bases 0x811C9DC5
 *    and 0x811C9DC5 ^ 0xA5A5A5A5), mod z; a neighbour whose two entries are
 *    both set counts as visited and is dropped, otherwise both are set.  The
 *    neighbours of a row are filtered in stored order (a neighbour sees the
 *    entries set by those before it).  False positives drop nodes that were
 *    never seen, so results differ from EXACT.  Device memory: 4*z bytes
 *    per resident wave (entries are 32-bit tags ordered by query, row and
 *    neighbour, which resolve the in-row order in one round trip), taken
 *    with the search workspace the first time.
 *  - SEEN: Algorithm 2's visited filter with no false positives: one bit
 *    per node and resident wave, tested and set by one atomic per
 *    neighbour while the neighbours are scored; a row whose neighbours
 *    were all seen skips the worklist rank and merge.  A seen node can only
 *    be in the worklist already or past its last entry (which never grows
 *    once the worklist is full), so results equal EXACT's, ids and
 *    distances.  Each query logs the ids it set (up to 8,192; past that it
 *    only tests) and clears their words at its end.  Device memory per
 *    resident wave: n/8 bytes (rounded up to 128) plus 32 KiB, taken with
 *    the search workspace the first time. */
#define BANG_FILTER_EXACT 0u
#define BANG_FILTER_BLOOM 1u
#define BANG_FILTER_SEEN 2u
#define BANG_BLOOM_Z 399887u

/* The re-rank sorts a query's expanded nodes in on-chip memory when they
 * fit there and otherwise selects them in device memory; this flag takes
 * the device-memory path always (same results; for testing it). */
#define BANG_SEARCH_RERANK_GLOBAL 1u

/* With BANG_FILTER_SEEN: each query stops setting bits once it has logged
 * 64 ids or more (the medoid and its first row or two) and from then on
 * only tests, as a query does once its log is full (same results; for
 * testing that path). */
#define BANG_SEARCH_SEEN_LOG_SHORT 2u

/* The exact-distance search without its seen-id cache (BANG_TABLE_EXACT):
 * every neighbour's base row is read (same results; for measuring the
 * cache). */
#define BANG_SEARCH_NO_SEEN_CACHE 4u

/* Table storage forms.  Both reduced forms are computed from the FP32
 * entries of the PQ table section, so they are deterministic:
 *  - F16: entry * 2^-k rounded to half (nearest, ties to even), k >= 0 the
 *    smallest that keeps the largest entry <= 65504; ADC = FP32 sum of the
 *    widened halves in subspace order.
 *  - U8: per subspace j, lo_j = min_c T[j][c]; inv = 255 / max_j range_j
 *    (FP32); entry = rint((T[j][c] - lo_j) * inv) in [0, 255]; ADC = exact
 *    integer sum of the m entries, ranked as FP32.
 * The re-rank stays exact in every form. */
#define BANG_TABLE_F32 0u
#define BANG_TABLE_F16 1u
#define BANG_TABLE_U8 2u
/* No PQ table: the paper's Exact-distance Version (section
 * "Implementation Variants").  The search ranks every node by its exact
 * squared distance to the query (the re-rank's distance, computed from the
 * base vectors in device memory) and there is no re-rank: the result is
 * the k first entries of the final worklist.  c_max is ignored.  With the
 * default visited filter each wave also keeps a cache of seen ids in
 * on-chip memory (direct-mapped, cleared per query, sized from the LDS the
 * wave's share leaves at the search's occupancy: 256 to 4096 ids, or none
 * at large L): a neighbour found
 * there was seen before in the query, which the set union would drop, so
 * its base row is not read.  Results are unchanged. */
#define BANG_TABLE_EXACT 3u

/* Build an index on the current HIP device: validates the description
 * (ids in range, no duplicate ids in a row, m | d, supported (m, d/m,
 * dtype)) and copies everything to device memory.  On success *out owns
 * the copies; release with bang_index_destroy.  Errors: EINVAL, ENOMEM,
 * EDEVICE, EUNSUPPORTED. */
int bang_index_create(const bang_index_desc* desc, bang_index** out);

/* Free an index and its workspace (NULL is a no-op).  Synchronises the
 * device first. */
int bang_index_destroy(bang_index* index);

/* Stage 1, the PQ distance table (section "Construction of PQDistTable in
 * Parallel"): tables_out[q][j][c] = sum_t (query[q][j*d/m+t] -
 * codebook[j][c][t])^2 for j < m, c < 256, FP32, no FMA, t ascending.
 * queries: device [nq][d] of the index dtype; tables_out: device
 * [nq][m][256] FP32.  nq = 0 is a no-op. */
int bang_build_pq_tables(bang_index* index, const void* queries, uint64_t nq,
                         float* tables_out, void* stream);

/* The precision form's table build (stage 1 by matrix cores): the same
 * tables with BF16 MFMA and FP32 accumulation.  tables_out[q][j][c] =
 * |q_j|^2 + |c_jc|^2 - 2 <bf16(q_j), bf16(c_jc)>, the squared norms summed
 * in FP32 from the unrounded coordinates in order, the inner product of
 * the coordinates rounded to bfloat16 (nearest, ties to even) by
 * v_mfma_f32_32x32x4_2b_bf16 (FP32 accumulation in the hardware's order).
 * Its error against the exact table is at most about 2^-6 sum_t |q_t c_t|
 * (bfloat16 rounding of both factors), so the search's ids can differ from
 * those of the FP32 tables where that moves a key.  Arguments as
 * bang_build_pq_tables; feed the result to bang_search through
 * bang_search_opts.tables. */
int bang_build_pq_tables_bf16(bang_index* index, const void* queries,
                              uint64_t nq, float* tables_out, void* stream);

/* Stages 1-3 (Algorithm 2 with the in-memory graph, then the re-rank of
 * section "Re-ranking"): for each query, greedy search from the medoid with
 * a worklist of L entries ordered by (PQ distance, id) until every entry
 * is expanded, then exact distances for the expanded nodes and the k
 * nearest by (exact distance, id).
 * queries: device [nq][d]; out_ids: device [nq][k] uint32; out_dists:
 * device [nq][k] FP32.  Rows with fewer than k candidates are padded with
 * (BANG_NONE, +inf).  Requires 1 <= k <= L <= BANG_MAX_L and k <= n.
 * opts may be NULL. */
int bang_search(bang_index* index, const void* queries, uint64_t nq,
                uint32_t k, uint32_t L, uint32_t* out_ids, float* out_dists,
                const bang_search_opts* opts, void* stream);

/* bang_search without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and validation as
 * bang_search; it calls no hipMalloc, hipFree or allocating routine.  Its
 * device memory is a file-scope array of 32 MiB per GPU (set up by
 * bang_index_create, held until the process ends): the launch counters and
 * 8 * iter_cap bytes of expanded-node keys per resident wave, so a launch
 * runs at most (32 MiB - 256) / (8 * iter_cap) waves (4 MiB keys: 1,364
 * waves at L = 768), fewer than bang_search when its occupancy allows
 * more; BANG_ENOMEM if one wave's keys do not fit.  The set-union filter
 * only (BANG_EUNSUPPORTED for BLOOM or SEEN).  Every call on a GPU shares
 * that GPU's array, which keeps the last call's contents: calls that
 * overlap in time on one GPU (other streams, other threads) race and must
 * be serialised by the caller. */
int bang_search_noalloc(bang_index* index, const void* queries, uint64_t nq,
                        uint32_t k, uint32_t L, uint32_t* out_ids,
                        float* out_dists, const bang_search_opts* opts,
                        void* stream);

/* Stage 3 alone: exact top-k over given candidates.  cand: device
 * [nq][c_max] uint32; BANG_NONE or ids >= n are padding and are skipped;
 * ids in a row must be distinct.  1 <= c_max <= 4096, 1 <= k <= 1024.
 * Output layout and padding as bang_search. */
int bang_rerank(bang_index* index, const void* queries, uint64_t nq,
                const uint32_t* cand, uint32_t c_max, uint32_t k,
                uint32_t* out_ids, float* out_dists, void* stream);

/* Roofline probe: reads nreads adjacency rows of the index, row i of the
 * sequence being splitmix64(seed + i) mod n, each the way the search reads
 * an expanded node's row: with the adjacency in device memory the packed
 * row's ids and codes (row_ids + R*m bytes, 16-byte loads), with a
 * host-resident adjacency the R ids across the host link (4-byte loads).
 * One wave per row, 32 waves per CU.  Nothing is computed from the data;
 * the bytes read per row go to *row_bytes_out (may be NULL), and the
 * caller times the launch on `stream`.  sink: device pointer to 8 bytes
 * the kernel may write.  Errors: EINVAL, EDEVICE. */
int bang_index_probe(bang_index* index, uint64_t nreads, uint64_t seed,
                     uint64_t* sink, uint32_t* row_bytes_out, void* stream);

/* Stop requests.  The paper's search is one long batched launch (10,000
 * queries, and the persistent launch of a large mixed batch runs for
 * seconds); a stop request lets the host end such a launch early without
 * losing the device: every wave of a search that carries it
 * (bang_search_opts.abort) reads it at each query's start and once every
 * 64 expansions, and leaves normally once it is set, so the stream and the
 * index stay usable.  The request is a word of page-locked host memory
 * mapped for the device (a read crosses the host link); bang_abort_set is
 * a plain host store and may be called from any thread while the search
 * runs.
 *  - create: allocates the request, cleared.  Errors: ENOMEM, EDEVICE.
 *  - destroy: frees it (NULL is a no-op); no search carrying it may still
 *    be running.
 *  - set: asks every search carrying it to stop.
 *  - clear: withdraws the request and forgets that a search stopped.
 *  - status: after the caller has synchronised the search's stream,
 *    BANG_EABORTED if a search carrying the request stopped a query
 *    because of it since the last clear, else BANG_OK (EINVAL for NULL). */
int bang_abort_create(bang_abort** out);
int bang_abort_destroy(bang_abort* ab);
int bang_abort_set(bang_abort* ab);
int bang_abort_clear(bang_abort* ab);
int bang_abort_status(const bang_abort* ab);

/* Message of the last failed call on this thread ("" if none). */
const char* bang_last_error(void);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching request loop over one index.  The paper
 * only batches (its experiments search a fixed batch); this is the form a
 * search service takes.  Requests of nq queries, each with its own k and
 * L, queue on the host.  A scheduler thread packs the oldest queued
 * requests, up to max_batch queries, into one mixed-batch search launch
 * (bang_search_opts.query_L / query_k) as soon as one of `slots` launch
 * slots is free; each slot owns a HIP stream, a search workspace and
 * pinned staging buffers, so batches on different slots overlap on the
 * device, and requests that arrive while others are being searched start
 * as soon as a slot frees up.  Every query's result is the one a search of
 * that query alone with the same (k, L) returns.  Results are copied back
 * to host memory.
 * ---------------------------------------------------------------------- */
typedef struct bang_server bang_server; /* opaque */

typedef struct {
  uint32_t max_batch;       /* queries per launch, 1..2^20; a request may
                               hold at most this many */
  uint32_t slots;           /* launches in flight at once, 1..8 */
  uint32_t max_k;           /* largest k of a request, <= max_L */
  uint32_t max_L;           /* largest L of a request, <= BANG_MAX_L */
  uint32_t table;           /* BANG_TABLE_* every request is searched with */
  uint64_t hbm_budget_bytes;/* 0, or a device-memory budget for the slots:
                               admission by footprint, fewer slots when
                               `slots` of them do not fit (ENOMEM if one
                               does not) */
  uint32_t flags;           /* 0, or BANG_SERVER_GRAPHS */
} bang_server_opts;

/* Each slot replays its batches from HIP graphs: the copies of the queries
 * and their (k, L) in, the search and the copies of the results out are
 * captured once per (batch size rounded up to a power of two, largest k,
 * largest L) and replayed; the rows past the batch are searched with
 * L = k = 1 and dropped.  Results are the same as without the flag. */
#define BANG_SERVER_GRAPHS 1u

/* Allocate the slots (device workspace and buffers, pinned host buffers)
 * and start the scheduler thread.  The index must outlive the server.
 * Errors: EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED. */
int bang_server_create(bang_index* index, const bang_server_opts* opts,
                       bang_server** out);

/* Finish every queued and running request, stop the scheduler and free
 * the slots (NULL is a no-op).  Results not yet collected are dropped. */
int bang_server_destroy(bang_server* server);

/* Queue a request: nq (1..max_batch) queries in HOST memory, copied before
 * the call returns, searched with 1 <= k <= L, k <= max_k, L <= max_L.
 * Never waits for the device.  *ticket names the request for
 * bang_server_wait.  Thread-safe. */
int bang_server_submit(bang_server* server, const void* queries, uint32_t nq,
                       uint32_t k, uint32_t L, uint64_t* ticket);

/* Wait for a request (timeout_ms < 0: without limit) and copy its results
 * to host ids[nq][k] / dists[nq][k] (either may be NULL), then forget the
 * ticket.  EABORTED on timeout (the request stays queued and the ticket
 * valid); a failed search returns its error.  Thread-safe. */
int bang_server_wait(bang_server* server, uint64_t ticket, uint32_t* ids,
                     float* dists, int timeout_ms);

/* Open-loop replay, for measurement: request j arrives arrival_s[j]
 * seconds after the call (non-decreasing) with nq[j] queries (the next
 * rows of `queries`, host memory), k[j] and L[j].  The call submits each
 * at its time, waits for all, and writes the results in request order to
 * host ids / dists with row stride kstride >= max k[j] (padded with
 * (BANG_NONE, +inf)) and latency_s[j] = completion time - arrival time
 * (-1 for a failed request; the first failure is returned). */
int bang_server_replay(bang_server* server, const void* queries,
                       uint32_t nreq, const uint32_t* nq, const uint32_t* k,
                       const uint32_t* L, const double* arrival_s,
                       uint32_t kstride, uint32_t* ids, float* dists,
                       double* latency_s);

/* Counters: {requests submitted, launches, queries launched, most slots
 * busy at once, slots}; the first n (<= 5) are written to out. */
int bang_server_stats(bang_server* server, uint64_t* out, uint32_t n);

#ifdef __cplusplus
}
#endif

#endif /* BANG_H_ */
