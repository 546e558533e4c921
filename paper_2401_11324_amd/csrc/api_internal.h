// Host-side state shared by the C ABI (bang_api.cpp) and the serving loop
// (bang_server.cpp): the index object, search workspaces, error reporting
// and the validated search entry.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "bang.h"
#include "internal.h"

namespace bang {

// Device memory one search launch needs besides its inputs and outputs:
// the expanded-node keys of every resident wave and the two counters of
// the persistent launch (zero between launches).  Launches that overlap in
// time need workspaces of their own.
struct Workspace {
  uint64_t* cscratch = nullptr;
  size_t cscratch_bytes = 0;
  uint32_t* qcounter = nullptr;
  // Bloom filter (BANG_FILTER_BLOOM only): BANG_BLOOM_Z entries and one
  // query epoch per resident wave, for bloom_waves waves
  uint32_t* bloom = nullptr;
  uint32_t* bloom_epoch = nullptr;
  uint64_t bloom_waves = 0;
  // seen bitmaps (BANG_FILTER_SEEN): per resident wave seen_words words
  // (zero between queries) and a log of seen_log_entries() ids, for
  // seen_waves waves
  uint32_t* seen = nullptr;
  uint32_t* seen_log = nullptr;
  uint32_t seen_words = 0;
  uint64_t seen_waves = 0;
  // true for a fixed workspace that limits the resident grid to what its
  // candidate buffer holds instead of failing (the no-allocation search)
  bool clamp_grid = false;
};

int workspace_init(Workspace* ws, size_t cscratch_bytes);
void workspace_free(Workspace* ws);

// Sets the thread-local error message and returns code.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
const char* last_error();

}  // namespace bang

// A stop request: two words of coherent, mapped, page-locked host memory,
// [0] the request (host writes, device reads) and [1] set by the device
// when a query stopped because of it.
struct bang_abort {
  uint32_t* host = nullptr;
  uint32_t* dev = nullptr;  // the same words as the device addresses them
};

struct bang_index {
  int device = 0;
  bang::DeviceIndex dev{};
  void* d_base = nullptr;
  unsigned char* d_rows = nullptr;
  uint32_t* h_adj = nullptr;  // pinned host adjacency (BANG_INDEX_HOST_ADJ)
  uint8_t* d_codes = nullptr;
  float* d_cb = nullptr;
  uint16_t* d_base16 = nullptr;  // bfloat16 base (BANG_INDEX_BF16_BASE)
  float* d_norm16 = nullptr;     // sums of squares of its rows
  bang::Workspace ws;         // used by bang_search; grown on demand
  int num_cus = 0;
  int max_lds = 64 * 1024;    // dynamic LDS bytes one workgroup may use
  int lds_per_cu = 64 * 1024; // LDS bytes of one CU
};

namespace bang {

// Workspace bytes a launch with these parameters needs (grid x iter_cap
// keys); 0 with an error set if the launch cannot run at all.
size_t search_workspace_bytes(bang_index* ix, uint64_t nq, uint32_t L,
                              uint32_t iter_cap, uint32_t table);

// Seen bitmaps for `grid` resident waves in ws (BANG_FILTER_SEEN),
// allocated and cleared when missing or too small; grow = false makes that
// an error instead.
int seen_reserve(bang_index* ix, Workspace* ws, bool grow, uint64_t grid);

// bang_search on an explicit workspace.  grow = false: a workspace that is
// too small is an error instead of being reallocated (reallocation
// synchronises the device).
int search_with(bang_index* ix, Workspace* ws, bool grow, const void* queries,
                uint64_t nq, uint32_t k, uint32_t L, uint32_t* out_ids,
                float* out_dists, const bang_search_opts* o, hipStream_t s);

}  // namespace bang
