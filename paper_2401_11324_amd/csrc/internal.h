// Internal interface between the C-ABI layer (bang_api.cpp) and the HIP
// kernels (bang_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bang {

enum Dtype : int { kF32 = 0, kU8 = 1, kI8 = 2 };

// Device copies of an index.
struct DeviceIndex {
  const void* base;           // [n][d]
  const unsigned char* rows;  // [n][row_stride_bytes]: ids, neighbour codes
                              // (null when the adjacency is host-resident)
  const uint32_t* hadj;       // [n][R] in pinned host memory, or null
  const uint8_t* codes;       // [n][m]
  const float* cb;            // [m][256][d/m]
  const uint16_t* base16;     // [n][d] float base rounded to bfloat16, or
                              // null (BANG_INDEX_BF16_BASE)
  const float* norm16;        // [n] sum of squares of each bfloat16 row
  uint32_t n, d, R, m, medoid;
  int dtype;
};

struct SearchLaunch {
  const void* queries;
  uint64_t nq;
  uint32_t k, L, c_max, iter_cap;
  int table;             // 0 FP32, 1 FP16, 2 U8 (bang_search_opts.table)
  bool rerank_bf16;      // BANG_RERANK_BF16 (float data, base16 present)
  uint32_t flags;        // bang_search_opts.flags
  uint32_t* out_ids;
  float* out_dists;
  const uint32_t* qL;    // per-query L / k (device, [nq]) or null
  const uint32_t* qk;
  uint32_t* out_cand;
  uint32_t cand_stride;
  uint32_t* out_counters;
  uint64_t* out_times;
  uint64_t* cscratch;    // [grid][iter_cap] expanded-node keys
  uint32_t* qcounter;    // [2]: next query, finished workgroups; zero
                         // between launches (the kernel resets them)
  uint32_t* out_phases;  // [nq][7] per-phase cycles (timed variant) or null
  uint32_t* bloom;       // null (exact filter) or [grid][BANG_BLOOM_Z]
  uint32_t* bloom_epoch; // [grid] query epoch of each wave's filter
  const float* tables;   // null, or [nq][m][256] FP32 tables to search by
                         // (instead of building them)
  const uint32_t* order;  // null, or [nq]: the order the waves take queries
  uint32_t* seen;        // null, or [grid][seen_words] seen bitmaps (zero
                         // between queries; BANG_FILTER_SEEN)
  uint32_t* seen_log;    // [grid][seen_log_entries()] ids set per query
  uint32_t seen_words;
  uint32_t seen_cap;     // ids a query may log (<= seen_log_entries())
  const uint32_t* abort_flag;  // device view of a bang_abort, or null
  uint32_t* abort_fired;
  uint32_t grid;         // workgroups (one wave each)
  uint32_t cache_slots;  // exact distances: seen-id cache entries per wave
                         // in LDS (0 or a power of two >= 256)
};

// The no-allocation search's device memory: a file-scope array of
// kNoallocScratchBytes per GPU (bang_kernels.hip).  setup looks its address
// up on `device`, which must be current, and zeroes the launch counters; it
// runs once per device (bang_index_create calls it).  noalloc_scratch
// returns that address, or null before the setup.
constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
hipError_t noalloc_scratch_setup(int device);
void* noalloc_scratch(int device);

// True if (dtype, m, d/m) has a compiled kernel.
bool supported(int dtype, uint32_t m, uint32_t dsub);

// LDS bytes the search kernel needs for a worklist of L, an iteration cap
// and a table storage form (a seen-id cache comes after them).
size_t search_lds_bytes(uint32_t m, uint32_t L, uint32_t iter_cap, int table);

// Packed adjacency rows: R ids padded to row_ids_bytes, then R x m codes.
uint32_t row_ids_bytes(uint32_t R);
uint32_t row_stride_bytes(uint32_t R, uint32_t m);
hipError_t launch_pack(const uint32_t* adj, const uint8_t* codes, uint32_t n,
                       uint32_t R, uint32_t m, unsigned char* rows,
                       hipStream_t s);

// Visited filter of a search variant: none (set union in the worklist),
// the paper's Bloom filter, or the exact seen bitmap.
enum FilterKind : int { kFilterUnion = 0, kFilterBloom = 1, kFilterSeen = 2 };

// Seen-bitmap words per resident wave for n nodes (one bit each, a whole
// number of 128-byte lines) and logged ids per wave.
uint32_t seen_words_for(uint32_t n);
uint32_t seen_log_entries();

// Resident workgroups per CU for the search kernel variant (adjacency
// placement of ix, visited filter, timed) at this LDS size.
hipError_t search_occupancy(const DeviceIndex& ix, int table, int filter,
                            bool phases, size_t lds, int* per_cu);

hipError_t launch_tables(const DeviceIndex& ix, const void* queries,
                         uint64_t nq, float* out, hipStream_t s);
// The same tables by BF16 MFMA with FP32 accumulation (bang.h
// bang_build_pq_tables_bf16).
hipError_t launch_tables_mfma(const DeviceIndex& ix, const void* queries,
                              uint64_t nq, float* out, hipStream_t s);
hipError_t launch_search(const DeviceIndex& ix, const SearchLaunch& a,
                         hipStream_t s);
// Random-row read probe over the index's adjacency (bang_index_probe);
// row_bytes receives the bytes read per row.
hipError_t launch_probe(const DeviceIndex& ix, uint64_t nreads, uint64_t seed,
                        uint64_t* sink, uint32_t grid, uint32_t* row_bytes,
                        hipStream_t s);

hipError_t launch_rerank(const DeviceIndex& ix, const void* queries,
                         uint64_t nq, const uint32_t* cand, uint32_t c_max,
                         uint32_t k, uint32_t* out_ids, float* out_dists,
                         hipStream_t s);

uint32_t pow2ceil(uint32_t x);

// The float base rounded to bfloat16 (nearest, ties to even) and the sum of
// squares of each rounded row (FP32, coordinates in order).
hipError_t launch_bf16_base(const float* base, uint64_t n, uint32_t d,
                            uint16_t* out16, float* norms, hipStream_t s);

}  // namespace bang
