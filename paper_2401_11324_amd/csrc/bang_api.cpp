// C ABI of the MI355X batched PQ graph search (see include/bang.h).
// Host-side validation, device copies of the index, workspace, launches.
// C++ exceptions never cross the ABI: every entry point catches them.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "api_internal.h"

namespace bang {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(BANG_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

int workspace_init(Workspace* ws, size_t cscratch_bytes) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&ws->qcounter),
                           2 * sizeof(uint32_t));
  if (e != hipSuccess) {
    ws->qcounter = nullptr;
    return fail(BANG_ENOMEM, std::string("search counters: ") +
                                 hipGetErrorString(e));
  }
  // the counters start at zero; every launch leaves them at zero
  e = hipMemset(ws->qcounter, 0, 2 * sizeof(uint32_t));
  if (e != hipSuccess) return hip_fail(e, "clearing the search counters");
  if (cscratch_bytes) {
    e = hipMalloc(reinterpret_cast<void**>(&ws->cscratch), cscratch_bytes);
    if (e != hipSuccess) {
      ws->cscratch = nullptr;
      return fail(BANG_ENOMEM, std::string("search workspace: ") +
                                   hipGetErrorString(e));
    }
    ws->cscratch_bytes = cscratch_bytes;
  }
  return BANG_OK;
}

void workspace_free(Workspace* ws) {
  (void)hipFree(ws->cscratch);
  (void)hipFree(ws->qcounter);
  (void)hipFree(ws->bloom);
  (void)hipFree(ws->bloom_epoch);
  (void)hipFree(ws->seen);
  (void)hipFree(ws->seen_log);
  *ws = Workspace{};
}

}  // namespace bang

using bang::fail;
using bang::hip_fail;

namespace {

size_t elem_size(int dt) { return dt == BANG_F32 ? 4 : 1; }

bool aligned(const void* p, size_t a) {
  return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

// Adjacency check: ids in range, no id twice in a row.  Rows are split
// across a few host threads.
bool check_adjacency(const uint32_t* adj, uint64_t n, uint32_t R,
                     std::string* why) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::string> errs(nt);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    th.emplace_back([&, t] {
      std::vector<uint32_t> row(R);
      for (uint64_t i = t; i < n && errs[t].empty(); i += nt) {
        uint32_t c = 0;
        for (uint32_t r = 0; r < R; ++r) {
          uint32_t x = adj[i * R + r];
          if (x == BANG_NONE) continue;
          if (x >= n) {
            errs[t] = "adjacency row " + std::to_string(i) + " holds id " +
                      std::to_string(x) + " >= n";
            return;
          }
          row[c++] = x;
        }
        std::sort(row.begin(), row.begin() + c);
        for (uint32_t r = 1; r < c; ++r)
          if (row[r] == row[r - 1]) {
            errs[t] = "adjacency row " + std::to_string(i) +
                      " holds id " + std::to_string(row[r]) + " twice";
            return;
          }
      }
    });
  }
  for (auto& x : th) x.join();
  for (auto& e : errs)
    if (!e.empty()) {
      *why = e;
      return false;
    }
  return true;
}

template <typename T>
int upload(T** dst, const void* src, size_t bytes, const char* what) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes ? bytes : 16);
  if (e != hipSuccess)
    return fail(BANG_ENOMEM, std::string("hipMalloc for ") + what + ": " +
                                 hipGetErrorString(e));
  if (bytes) {
    e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
  }
  return BANG_OK;
}

void free_index(bang_index* ix) {
  if (!ix) return;
  (void)hipFree(ix->d_base);
  (void)hipFree(ix->d_rows);
  if (ix->h_adj) (void)hipHostFree(ix->h_adj);
  (void)hipFree(ix->d_codes);
  (void)hipFree(ix->d_cb);
  (void)hipFree(ix->d_base16);
  (void)hipFree(ix->d_norm16);
  bang::workspace_free(&ix->ws);
  delete ix;
}

int create_impl(const bang_index_desc* d, bang_index** out) {
  if (!d || !out) return fail(BANG_EINVAL, "null argument");
  *out = nullptr;
  if (d->flags & ~(BANG_INDEX_HOST_ADJ | BANG_INDEX_BF16_BASE))
    return fail(BANG_EINVAL, "unknown index flags");
  if ((d->flags & BANG_INDEX_BF16_BASE) &&
      (d->dtype != BANG_F32 || d->d % 8 != 0))
    return fail(BANG_EUNSUPPORTED,
                "BANG_INDEX_BF16_BASE needs float data with d a multiple "
                "of 8");
  if (d->n == 0 || d->n >= (1ull << 31))
    return fail(BANG_EINVAL, "n must be in [1, 2^31)");
  if (d->dtype < BANG_F32 || d->dtype > BANG_I8)
    return fail(BANG_EINVAL, "unknown dtype");
  if (d->d == 0 || d->m == 0 || d->d % d->m != 0)
    return fail(BANG_EINVAL, "m must divide d");
  if (d->R == 0 || d->R > BANG_MAX_R)
    return fail(BANG_EINVAL, "R must be in [1, 64]");
  if (d->medoid >= d->n) return fail(BANG_EINVAL, "medoid >= n");
  if (!d->base || !d->adj || !d->codebooks || !d->codes)
    return fail(BANG_EINVAL, "null array in the description");
  if (!bang::supported(d->dtype, d->m, d->d / d->m))
    return fail(BANG_EUNSUPPORTED,
                "no kernel for dtype " + std::to_string(d->dtype) + ", m=" +
                    std::to_string(d->m) + ", d/m=" +
                    std::to_string(d->d / d->m));
  std::string why;
  if (!check_adjacency(d->adj, d->n, d->R, &why)) return fail(BANG_EINVAL, why);

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0)
    return fail(BANG_EDEVICE, "no HIP device available");
  auto* ix = new (std::nothrow) bang_index();
  if (!ix) return fail(BANG_ENOMEM, "host allocation");
  e = hipGetDevice(&ix->device);
  if (e != hipSuccess) {
    delete ix;
    return hip_fail(e, "hipGetDevice");
  }
  e = hipDeviceGetAttribute(&ix->num_cus, hipDeviceAttributeMultiprocessorCount,
                            ix->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&ix->max_lds,
                              hipDeviceAttributeMaxSharedMemoryPerBlock,
                              ix->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&ix->lds_per_cu,
                              hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              ix->device);
  if (e != hipSuccess) {
    delete ix;
    return hip_fail(e, "hipDeviceGetAttribute");
  }
  int rc;
  size_t nd = (size_t)d->n * d->d;
  const bool host_adj = (d->flags & BANG_INDEX_HOST_ADJ) != 0;
  const size_t adj_bytes = (size_t)d->n * d->R * 4;
  uint32_t* d_adj = nullptr;
  if ((rc = upload(&ix->d_base, d->base, nd * elem_size(d->dtype), "base")) ||
      (!host_adj &&
       (rc = upload(&d_adj, d->adj, adj_bytes, "adjacency"))) ||
      (rc = upload(&ix->d_codes, d->codes, (size_t)d->n * d->m, "codes")) ||
      (rc = upload(&ix->d_cb, d->codebooks, (size_t)d->m * 256 * (d->d / d->m) * 4,
                   "codebooks")) ||
      (rc = bang::workspace_init(&ix->ws, 0))) {
    (void)hipFree(d_adj);
    free_index(ix);
    return rc;
  }
  if (host_adj) {
    // page-locked, GPU-cacheable (the kernels only read it), mapped into
    // the device address space
    e = hipHostMalloc(reinterpret_cast<void**>(&ix->h_adj), adj_bytes,
                      hipHostMallocNonCoherent);
    if (e != hipSuccess) {
      ix->h_adj = nullptr;
      free_index(ix);
      return fail(BANG_ENOMEM, std::string("pinned host adjacency: ") +
                                   hipGetErrorString(e));
    }
    std::memcpy(ix->h_adj, d->adj, adj_bytes);
    void* dptr = nullptr;
    e = hipHostGetDevicePointer(&dptr, ix->h_adj, 0);
    if (e != hipSuccess) {
      free_index(ix);
      return hip_fail(e, "hipHostGetDevicePointer");
    }
    ix->dev.hadj = static_cast<const uint32_t*>(dptr);
    ix->dev.rows = nullptr;
  }
  // rows: each node's adjacency followed by its neighbours' codes, so one
  // coalesced load per expansion brings both (layout in internal.h)
  const size_t row_bytes = (size_t)d->n * bang::row_stride_bytes(d->R, d->m);
  if (!host_adj) {
    e = hipMalloc(reinterpret_cast<void**>(&ix->d_rows), row_bytes);
    if (e != hipSuccess) {
      (void)hipFree(d_adj);
      free_index(ix);
      return fail(BANG_ENOMEM, std::string("hipMalloc for packed rows: ") +
                                   hipGetErrorString(e));
    }
    e = hipMemset(ix->d_rows, 0, row_bytes);
  }
  if (e == hipSuccess && !host_adj)
    e = bang::launch_pack(d_adj, ix->d_codes, (uint32_t)d->n, d->R, d->m,
                          ix->d_rows, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(d_adj);
  if (e != hipSuccess) {
    free_index(ix);
    return hip_fail(e, "packing adjacency rows");
  }
  ix->dev.base = ix->d_base;
  if (!host_adj) ix->dev.rows = ix->d_rows;
  ix->dev.codes = ix->d_codes;
  ix->dev.cb = ix->d_cb;
  if (d->flags & BANG_INDEX_BF16_BASE) {
    e = hipMalloc(reinterpret_cast<void**>(&ix->d_base16), nd * 2);
    if (e == hipSuccess)
      e = hipMalloc(reinterpret_cast<void**>(&ix->d_norm16), d->n * 4);
    if (e != hipSuccess) {
      free_index(ix);
      return fail(BANG_ENOMEM, std::string("bfloat16 base: ") +
                                   hipGetErrorString(e));
    }
    e = bang::launch_bf16_base(static_cast<const float*>(ix->d_base), d->n,
                               d->d, ix->d_base16, ix->d_norm16, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      free_index(ix);
      return hip_fail(e, "bfloat16 base");
    }
    ix->dev.base16 = ix->d_base16;
    ix->dev.norm16 = ix->d_norm16;
  }
  ix->dev.n = (uint32_t)d->n;
  ix->dev.d = d->d;
  ix->dev.R = d->R;
  ix->dev.m = d->m;
  ix->dev.medoid = d->medoid;
  ix->dev.dtype = d->dtype;
  // the no-allocation search's device memory on this GPU, found once
  e = bang::noalloc_scratch_setup(ix->device);
  if (e != hipSuccess) {
    free_index(ix);
    return hip_fail(e, "no-allocation scratch set-up");
  }
  *out = ix;
  return BANG_OK;
}

int check_queries(const bang_index* ix, const void* queries) {
  if (!queries) return fail(BANG_EINVAL, "null queries");
  if (!aligned(queries, 16)) return fail(BANG_EINVAL, "queries not 16-byte aligned");
  if ((ix->dev.d * elem_size(ix->dev.dtype)) % 16 != 0)
    return fail(BANG_EUNSUPPORTED, "query rows must be a multiple of 16 bytes");
  return BANG_OK;
}

// Launch geometry of a search: LDS bytes and resident workgroups.
// LDS bytes, resident waves and, for the exact-distance search with the set
// union (unless no_cache), the seen-id cache's slots: the largest power of
// two from 256 to kCacheMaxSlots whose LDS still leaves the occupancy the
// search has without it (0 if none does).
constexpr uint32_t kCacheMaxSlots = 4096;

int search_geometry(bang_index* ix, uint64_t nq, uint32_t L, uint32_t iter_cap,
                    uint32_t table, int filter, bool phases, size_t* lds,
                    uint64_t* grid, uint32_t waves_per_cu = 0,
                    uint32_t* cache_slots = nullptr, bool no_cache = false) {
  if (cache_slots) *cache_slots = 0;
  *lds = bang::search_lds_bytes(ix->dev.m, L, iter_cap, (int)table);
  hipError_t e = hipSetDevice(ix->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (*lds > (size_t)ix->max_lds)
    return fail(BANG_EUNSUPPORTED,
                "table + worklist + re-rank keys need " + std::to_string(*lds) +
                    " bytes of LDS, the device allows " +
                    std::to_string(ix->max_lds) + " (lower L or iter_cap)");
  int per_cu = 0;
  e = bang::search_occupancy(ix->dev, (int)table, filter, phases, *lds,
                             &per_cu);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  if (per_cu < 1) return fail(BANG_EUNSUPPORTED, "search kernel cannot be resident");
  if (waves_per_cu) per_cu = std::min<int>(per_cu, (int)waves_per_cu);
  if (cache_slots && !no_cache && table == BANG_TABLE_EXACT &&
      filter == bang::kFilterUnion) {
    const size_t share = (size_t)ix->lds_per_cu / (size_t)per_cu;
    for (uint32_t c = kCacheMaxSlots; c >= 256; c >>= 1) {
      const size_t with = *lds + 4 * (size_t)c;
      if (with > share || with > (size_t)ix->max_lds) continue;
      int pc = 0;
      e = bang::search_occupancy(ix->dev, (int)table, filter, phases, with,
                                 &pc);
      if (e != hipSuccess) return hip_fail(e, "occupancy query");
      if (pc >= per_cu) {
        *cache_slots = c;
        *lds = with;
        break;
      }
    }
  }
  *grid = std::min<uint64_t>((uint64_t)per_cu * ix->num_cus, nq);
  return BANG_OK;
}

}  // namespace

namespace bang {

size_t search_workspace_bytes(bang_index* ix, uint64_t nq, uint32_t L,
                              uint32_t iter_cap, uint32_t table) {
  size_t lds;
  uint64_t grid;
  if (search_geometry(ix, nq, L, iter_cap, table, kFilterUnion, false, &lds,
                      &grid))
    return 0;
  return (size_t)grid * iter_cap * sizeof(uint64_t);
}

// Seen bitmaps and logs for `grid` waves in ws, allocated (and cleared)
// the first time or when a launch needs more waves (grow only).
int seen_reserve(bang_index* ix, Workspace* ws, bool grow, uint64_t grid) {
  const uint32_t words = seen_words_for(ix->dev.n);
  if (grid <= ws->seen_waves && ws->seen_words >= words) return BANG_OK;
  if (!grow)
    return fail(BANG_ENOMEM, "seen bitmaps for " +
                                 std::to_string(ws->seen_waves) +
                                 " waves, the launch needs " +
                                 std::to_string(grid));
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  (void)hipFree(ws->seen);
  (void)hipFree(ws->seen_log);
  ws->seen = ws->seen_log = nullptr;
  ws->seen_waves = 0;
  ws->seen_words = 0;
  const size_t bb = (size_t)grid * words * sizeof(uint32_t);
  const size_t lb = (size_t)grid * seen_log_entries() * sizeof(uint32_t);
  e = hipMalloc(reinterpret_cast<void**>(&ws->seen), bb);
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void**>(&ws->seen_log), lb);
  if (e != hipSuccess) {
    (void)hipFree(ws->seen);
    ws->seen = nullptr;
    return fail(BANG_ENOMEM,
                std::string("seen bitmaps: ") + hipGetErrorString(e));
  }
  // every bit clear; each query leaves the bits it set clear again
  e = hipMemset(ws->seen, 0, bb);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "seen bitmap init");
  ws->seen_waves = grid;
  ws->seen_words = words;
  return BANG_OK;
}

int search_with(bang_index* ix, Workspace* ws, bool grow, const void* queries,
                uint64_t nq, uint32_t k, uint32_t L, uint32_t* out_ids,
                float* out_dists, const bang_search_opts* o, hipStream_t s) {
  if (!ix) return fail(BANG_EINVAL, "null index");
  if (k < 1 || k > L || L > BANG_MAX_L)
    return fail(BANG_EINVAL, "need 1 <= k <= L <= 1024");
  if (k > ix->dev.n) return fail(BANG_EINVAL, "k > n");
  if (nq == 0) return BANG_OK;
  if (nq >= (1ull << 32)) return fail(BANG_EINVAL, "nq too large");
  int rc = check_queries(ix, queries);
  if (rc) return rc;
  if (!out_ids || !out_dists) return fail(BANG_EINVAL, "null output");
  if (!aligned(out_ids, 4) || !aligned(out_dists, 4))
    return fail(BANG_EINVAL, "outputs not 4-byte aligned");
  const bool mixed = o && (o->query_L || o->query_k);
  if (mixed && (o->c_max || o->iter_cap))
    return fail(BANG_EINVAL,
                "a mixed batch (query_L / query_k) takes the default c_max "
                "and iter_cap of each query's L");
  if (o && ((o->query_L && !aligned(o->query_L, 4)) ||
            (o->query_k && !aligned(o->query_k, 4))))
    return fail(BANG_EINVAL, "query_L / query_k not 4-byte aligned");
  uint32_t c_max = (o && o->c_max) ? o->c_max : 4 * L;
  uint32_t iter_cap = (o && o->iter_cap) ? o->iter_cap : std::max(4 * L, L + 64);
  const uint32_t table = o ? o->table : BANG_TABLE_F32;
  if (table > BANG_TABLE_EXACT) return fail(BANG_EINVAL, "unknown table form");
  if (iter_cap > 8192) return fail(BANG_EINVAL, "iter_cap > 8192");
  if (o && o->out_cand && o->cand_stride == 0)
    return fail(BANG_EINVAL, "cand_stride must be > 0 with out_cand");
  const uint32_t flags = o ? o->flags : 0u;
  if (flags & ~(BANG_SEARCH_RERANK_GLOBAL | BANG_SEARCH_SEEN_LOG_SHORT |
                BANG_SEARCH_NO_SEEN_CACHE))
    return fail(BANG_EINVAL, "unknown search flags");
  const uint32_t filter = o ? o->filter : BANG_FILTER_EXACT;
  if (filter > BANG_FILTER_SEEN)
    return fail(BANG_EINVAL, "unknown visited filter");
  const int fkind = filter == BANG_FILTER_BLOOM
                        ? bang::kFilterBloom
                        : (filter == BANG_FILTER_SEEN ? bang::kFilterSeen
                                                      : bang::kFilterUnion);
  const uint32_t rerank = o ? o->rerank : BANG_RERANK_EXACT;
  if (rerank > BANG_RERANK_BF16) return fail(BANG_EINVAL, "unknown re-rank");
  if (rerank == BANG_RERANK_BF16 && !ix->dev.base16)
    return fail(BANG_EINVAL,
                "BANG_RERANK_BF16 needs an index created with "
                "BANG_INDEX_BF16_BASE");
  if (rerank == BANG_RERANK_BF16 && table == BANG_TABLE_EXACT)
    return fail(BANG_EINVAL,
                "the exact-distance search has no re-rank to make BF16");
  const float* const tables = o ? o->tables : nullptr;
  if (tables && table == BANG_TABLE_EXACT)
    return fail(BANG_EINVAL,
                "the exact-distance search has no table to take (tables)");
  if (tables && !aligned(tables, 4))
    return fail(BANG_EINVAL, "tables not 4-byte aligned");

  size_t lds;
  uint64_t grid;
  uint32_t* const phases = o ? o->out_phases : nullptr;
  if (phases && (ix->dev.hadj || filter == BANG_FILTER_BLOOM))
    return fail(BANG_EUNSUPPORTED,
                "out_phases: the timed search has the device-resident "
                "adjacency and no Bloom filter");
  if (phases && !aligned(phases, 4))
    return fail(BANG_EINVAL, "out_phases not 4-byte aligned");
  const uint32_t* const order = o ? o->order : nullptr;
  if (order && !aligned(order, 4))
    return fail(BANG_EINVAL, "order not 4-byte aligned");
  uint32_t cache_slots = 0;
  rc = search_geometry(ix, nq, L, iter_cap, table, fkind, phases != nullptr,
                       &lds, &grid, o ? o->waves_per_cu : 0u, &cache_slots,
                       (flags & BANG_SEARCH_NO_SEEN_CACHE) != 0);
  if (rc) return rc;
  size_t need = (size_t)grid * iter_cap * sizeof(uint64_t);
  if (need > ws->cscratch_bytes && ws->clamp_grid) {
    // fewer resident waves, each with its whole candidate buffer
    grid = ws->cscratch_bytes / ((size_t)iter_cap * sizeof(uint64_t));
    if (grid == 0)
      return fail(BANG_ENOMEM,
                  "the no-allocation scratch (" +
                      std::to_string(ws->cscratch_bytes) +
                      " bytes of candidates) holds no wave of " +
                      std::to_string(iter_cap) + " iterations");
    need = (size_t)grid * iter_cap * sizeof(uint64_t);
  }
  if (need > ws->cscratch_bytes) {
    if (!grow)
      return fail(BANG_ENOMEM, "search workspace of " +
                                   std::to_string(ws->cscratch_bytes) +
                                   " bytes, the launch needs " +
                                   std::to_string(need));
    // the previous workspace may still be in use by queued work
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    (void)hipFree(ws->cscratch);
    ws->cscratch = nullptr;
    ws->cscratch_bytes = 0;
    e = hipMalloc(reinterpret_cast<void**>(&ws->cscratch), need);
    if (e != hipSuccess)
      return fail(BANG_ENOMEM, std::string("search workspace: ") +
                                   hipGetErrorString(e));
    ws->cscratch_bytes = need;
  }
  if (filter == BANG_FILTER_BLOOM && grid > ws->bloom_waves) {
    if (!grow)
      return fail(BANG_ENOMEM, "Bloom filters for " +
                                   std::to_string(ws->bloom_waves) +
                                   " waves, the launch needs " +
                                   std::to_string(grid));
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    (void)hipFree(ws->bloom);
    (void)hipFree(ws->bloom_epoch);
    ws->bloom = ws->bloom_epoch = nullptr;
    ws->bloom_waves = 0;
    const size_t fb = (size_t)grid * BANG_BLOOM_Z * sizeof(uint32_t);
    e = hipMalloc(reinterpret_cast<void**>(&ws->bloom), fb);
    if (e == hipSuccess)
      e = hipMalloc(reinterpret_cast<void**>(&ws->bloom_epoch),
                    (size_t)grid * sizeof(uint32_t));
    if (e != hipSuccess) {
      (void)hipFree(ws->bloom);
      ws->bloom = nullptr;
      return fail(BANG_ENOMEM, std::string("Bloom filters: ") +
                                   hipGetErrorString(e));
    }
    // every entry unset (above any tag) and every epoch at its start
    e = hipMemset(ws->bloom, 0xFF, fb);
    if (e == hipSuccess)
      e = hipMemset(ws->bloom_epoch, 0, (size_t)grid * sizeof(uint32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "Bloom filter init");
    ws->bloom_waves = grid;
  }
  if (filter == BANG_FILTER_SEEN) {
    rc = seen_reserve(ix, ws, grow, grid);
    if (rc) return rc;
  }

  bang::SearchLaunch l{};
  l.queries = queries;
  l.nq = nq;
  l.k = k;
  l.L = L;
  l.c_max = c_max;
  l.iter_cap = iter_cap;
  l.table = (int)table;
  l.rerank_bf16 = rerank == BANG_RERANK_BF16;
  l.flags = flags;
  l.out_ids = out_ids;
  l.out_dists = out_dists;
  l.qL = o ? o->query_L : nullptr;
  l.qk = o ? o->query_k : nullptr;
  l.out_cand = o ? o->out_cand : nullptr;
  l.cand_stride = o ? o->cand_stride : 0;
  l.out_counters = o ? o->out_counters : nullptr;
  l.out_times = o ? o->out_times : nullptr;
  l.out_phases = phases;
  l.cscratch = ws->cscratch;
  l.qcounter = ws->qcounter;
  l.tables = tables;
  l.order = order;
  l.bloom = filter == BANG_FILTER_BLOOM ? ws->bloom : nullptr;
  l.bloom_epoch = filter == BANG_FILTER_BLOOM ? ws->bloom_epoch : nullptr;
  if (filter == BANG_FILTER_SEEN) {
    l.seen = ws->seen;
    l.seen_log = ws->seen_log;
    l.seen_words = ws->seen_words;
    l.seen_cap = (flags & BANG_SEARCH_SEEN_LOG_SHORT) ? 2u * 64u
                                                      : bang::seen_log_entries();
  }
  if (o && o->abort) {
    l.abort_flag = o->abort->dev;
    l.abort_fired = o->abort->dev + 1;
  }
  l.grid = (uint32_t)grid;
  l.cache_slots = cache_slots;
  hipError_t e = bang::launch_search(ix->dev, l, s);
  if (e != hipSuccess) return hip_fail(e, "search launch");
  return BANG_OK;
}

}  // namespace bang

namespace {
}  // namespace

extern "C" {

int bang_index_create(const bang_index_desc* desc, bang_index** out) {
  try {
    return create_impl(desc, out);
  } catch (const std::exception& ex) {
    return fail(BANG_ENOMEM, ex.what());
  } catch (...) {
    return fail(BANG_ENOMEM, "unknown exception");
  }
}

int bang_index_destroy(bang_index* index) {
  if (!index) return BANG_OK;
  (void)hipSetDevice(index->device);
  (void)hipDeviceSynchronize();
  free_index(index);
  return BANG_OK;
}

int bang_build_pq_tables(bang_index* ix, const void* queries, uint64_t nq,
                         float* tables_out, void* stream) {
  try {
    if (!ix) return fail(BANG_EINVAL, "null index");
    if (nq == 0) return BANG_OK;
    int rc = check_queries(ix, queries);
    if (rc) return rc;
    if (!tables_out || !aligned(tables_out, 16))
      return fail(BANG_EINVAL, "tables_out null or not 16-byte aligned");
    hipError_t e = hipSetDevice(ix->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = bang::launch_tables(ix->dev, queries, nq, tables_out,
                            static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "table launch");
    return BANG_OK;
  } catch (...) {
    return fail(BANG_ENOMEM, "exception");
  }
}

int bang_build_pq_tables_bf16(bang_index* ix, const void* queries,
                              uint64_t nq, float* tables_out, void* stream) {
  try {
    if (!ix) return fail(BANG_EINVAL, "null index");
    if (nq == 0) return BANG_OK;
    int rc = check_queries(ix, queries);
    if (rc) return rc;
    if (!tables_out || !aligned(tables_out, 16))
      return fail(BANG_EINVAL, "tables_out null or not 16-byte aligned");
    if (ix->dev.d / ix->dev.m > 8)
      return fail(BANG_EUNSUPPORTED, "d/m above 8");
    hipError_t e = hipSetDevice(ix->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = bang::launch_tables_mfma(ix->dev, queries, nq, tables_out,
                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "BF16 MFMA table launch");
    return BANG_OK;
  } catch (...) {
    return fail(BANG_ENOMEM, "exception");
  }
}

int bang_search(bang_index* ix, const void* queries, uint64_t nq, uint32_t k,
                uint32_t L, uint32_t* out_ids, float* out_dists,
                const bang_search_opts* opts, void* stream) {
  try {
    if (!ix) return fail(BANG_EINVAL, "null index");
    return bang::search_with(ix, &ix->ws, true, queries, nq, k, L, out_ids,
                             out_dists, opts, static_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(BANG_ENOMEM, "exception");
  }
}

int bang_search_noalloc(bang_index* ix, const void* queries, uint64_t nq,
                        uint32_t k, uint32_t L, uint32_t* out_ids,
                        float* out_dists, const bang_search_opts* opts,
                        void* stream) {
  try {
    if (!ix) return fail(BANG_EINVAL, "null index");
    if (opts && opts->filter != BANG_FILTER_EXACT)
      return fail(BANG_EUNSUPPORTED,
                  "the no-allocation search has the set-union filter only");
    void* p = bang::noalloc_scratch(ix->device);
    if (!p) return fail(BANG_EDEVICE, "no-allocation scratch not set up");
    bang::Workspace ws;
    ws.qcounter = static_cast<uint32_t*>(p);
    ws.cscratch = reinterpret_cast<uint64_t*>(static_cast<char*>(p) + 256);
    ws.cscratch_bytes = bang::kNoallocScratchBytes - 256;
    ws.clamp_grid = true;
    return bang::search_with(ix, &ws, false, queries, nq, k, L, out_ids,
                             out_dists, opts, static_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(BANG_ENOMEM, "exception");
  }
}

int bang_rerank(bang_index* ix, const void* queries, uint64_t nq,
                const uint32_t* cand, uint32_t c_max, uint32_t k,
                uint32_t* out_ids, float* out_dists, void* stream) {
  try {
    if (!ix) return fail(BANG_EINVAL, "null index");
    if (c_max < 1 || c_max > 4096) return fail(BANG_EINVAL, "need 1 <= c_max <= 4096");
    if (k < 1 || k > 1024) return fail(BANG_EINVAL, "need 1 <= k <= 1024");
    if (nq == 0) return BANG_OK;
    int rc = check_queries(ix, queries);
    if (rc) return rc;
    if (!cand || !out_ids || !out_dists || !aligned(cand, 4) ||
        !aligned(out_ids, 4) || !aligned(out_dists, 4))
      return fail(BANG_EINVAL, "null or misaligned buffer");
    hipError_t e = hipSetDevice(ix->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = bang::launch_rerank(ix->dev, queries, nq, cand, c_max, k, out_ids,
                            out_dists, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "re-rank launch");
    return BANG_OK;
  } catch (...) {
    return fail(BANG_ENOMEM, "exception");
  }
}

int bang_index_probe(bang_index* ix, uint64_t nreads, uint64_t seed,
                     uint64_t* sink, uint32_t* row_bytes_out, void* stream) {
  try {
    if (!ix) return fail(BANG_EINVAL, "null index");
    if (!sink || !aligned(sink, 8))
      return fail(BANG_EINVAL, "sink null or not 8-byte aligned");
    hipError_t e = hipSetDevice(ix->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    uint32_t rb = 0;
    e = bang::launch_probe(ix->dev, nreads, seed, sink,
                           (uint32_t)ix->num_cus * 8u, &rb,
                           static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "probe launch");
    if (row_bytes_out) *row_bytes_out = rb;
    return BANG_OK;
  } catch (...) {
    return fail(BANG_ENOMEM, "exception");
  }
}

int bang_abort_create(bang_abort** out) {
  try {
    if (!out) return fail(BANG_EINVAL, "null argument");
    *out = nullptr;
    auto* ab = new (std::nothrow) bang_abort();
    if (!ab) return fail(BANG_ENOMEM, "host allocation");
    // coherent: the device's reads and writes bypass its caches, so a host
    // store is seen by the next reading and the device's store by the host
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&ab->host),
                                 2 * sizeof(uint32_t),
                                 hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) {
      delete ab;
      return fail(BANG_ENOMEM, std::string("stop request: ") +
                                   hipGetErrorString(e));
    }
    __atomic_store_n(&ab->host[0], 0u, __ATOMIC_SEQ_CST);
    __atomic_store_n(&ab->host[1], 0u, __ATOMIC_SEQ_CST);
    void* dptr = nullptr;
    e = hipHostGetDevicePointer(&dptr, ab->host, 0);
    if (e != hipSuccess) {
      (void)hipHostFree(ab->host);
      delete ab;
      return hip_fail(e, "hipHostGetDevicePointer");
    }
    ab->dev = static_cast<uint32_t*>(dptr);
    *out = ab;
    return BANG_OK;
  } catch (...) {
    return fail(BANG_ENOMEM, "exception");
  }
}

int bang_abort_destroy(bang_abort* ab) {
  if (!ab) return BANG_OK;
  (void)hipHostFree(ab->host);
  delete ab;
  return BANG_OK;
}

int bang_abort_set(bang_abort* ab) {
  if (!ab) return fail(BANG_EINVAL, "null stop request");
  __atomic_store_n(&ab->host[0], 1u, __ATOMIC_SEQ_CST);
  return BANG_OK;
}

int bang_abort_clear(bang_abort* ab) {
  if (!ab) return fail(BANG_EINVAL, "null stop request");
  __atomic_store_n(&ab->host[0], 0u, __ATOMIC_SEQ_CST);
  __atomic_store_n(&ab->host[1], 0u, __ATOMIC_SEQ_CST);
  return BANG_OK;
}

int bang_abort_status(const bang_abort* ab) {
  if (!ab) return fail(BANG_EINVAL, "null stop request");
  if (__atomic_load_n(&ab->host[1], __ATOMIC_SEQ_CST))
    return fail(BANG_EABORTED, "a search stopped on the stop request");
  return BANG_OK;
}

const char* bang_last_error(void) { return bang::last_error(); }

}  // extern "C"
