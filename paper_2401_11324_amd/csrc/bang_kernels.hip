// HIP kernels for gfx950 (MI355X) besides the search (search_kernel.h,
// search_variants.hip): the stand-alone PQ table and re-rank kernels, the
// packing of adjacency rows with their neighbours' codes, and the host side
// of every launch (LDS sizes, occupancy, variant choice).

#include "search_kernel.h"

#include <mutex>

namespace bang {

// Device memory of the no-allocation search (bang_search_noalloc): the two
// launch counters in the first 256 bytes, then the expanded-node keys of
// every resident wave.  Each GPU the library runs on holds its own copy
// until the process ends; calls that overlap in time on one GPU share it
// and race.  Host code addresses it only through the device pointer that
// noalloc_scratch looked up for that GPU (the array's name is a host-side
// stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices];  // device address per GPU, once looked up
}  // namespace

hipError_t noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_at[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // caller sets it current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  // the counters start at zero (every search launch leaves them at zero)
  e = hipMemset(p, 0, 256);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  g_scratch_at[device] = p;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_at[device];
}

namespace {

// Packed rows: row u = R neighbour ids (padded to row_ids bytes), then the
// m code bytes of each neighbour slot (zero for an empty slot).
__global__ __launch_bounds__(256) void pack_rows_kernel(
    const uint32_t* __restrict__ adj, const uint8_t* __restrict__ codes,
    uint32_t n, uint32_t R, uint32_t m, uint32_t row_ids, uint32_t stride,
    unsigned char* __restrict__ out) {
  const uint64_t total = (uint64_t)n * R;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t u = t / R;
    const uint32_t r = (uint32_t)(t % R);
    const uint32_t id = adj[t];
    unsigned char* row = out + u * stride;
    reinterpret_cast<uint32_t*>(row)[r] = id;
    uint4* dst = reinterpret_cast<uint4*>(row + row_ids + (size_t)r * m);
    if (id != kNone) {
      const uint4* src = reinterpret_cast<const uint4*>(codes + (size_t)id * m);
      for (uint32_t i = 0; i < m / 16; ++i) dst[i] = src[i];
    } else {
      for (uint32_t i = 0; i < m / 16; ++i) dst[i] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

template <int DT, int M, int DS>
__global__ __launch_bounds__(256) void table_kernel(
    const unsigned char* __restrict__ queries, uint64_t nq,
    const float* __restrict__ cb, float* __restrict__ out) {
  constexpr int D = M * DS;
  for (uint64_t qi = blockIdx.x; qi < nq; qi += gridDim.x)
    build_table<DT, M, DS>(queries + qi * D * Elem<DT>::size, cb,
                           out + qi * (uint64_t)M * 256, threadIdx.x, 256);
}

template <int DT, int D>
__global__ __launch_bounds__(kWave) void rerank_kernel(
    const void* __restrict__ base, uint32_t n,
    const unsigned char* __restrict__ queries, uint64_t nq,
    const uint32_t* __restrict__ cand, uint32_t c_max, uint32_t k,
    uint32_t* out_ids, float* out_d) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* S = reinterpret_cast<uint64_t*>(smem);
  const int lane = threadIdx.x;
  for (uint64_t qi = blockIdx.x; qi < nq; qi += gridDim.x) {
    const unsigned char* q = queries + qi * D * Elem<DT>::size;
    const int32_t qq = query_sq<DT, D>(q);
    uint32_t cnt = 0;
    for (uint32_t i0 = 0; i0 < c_max; i0 += kWave) {
      uint32_t i = i0 + lane;
      uint32_t id = i < c_max ? cand[qi * c_max + i] : kNone;
      bool ok = id != kNone && id < n;
      uint64_t m = __ballot(ok);
      uint32_t idx = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      if (ok) S[cnt + idx] = make_key(exact_dist<DT, D>(base, id, q, qq), id);
      cnt += __popcll(m);
    }
    __syncthreads();
    sort_and_emit(S, cnt, k, out_ids + qi * k, out_d + qi * k, lane);
    __syncthreads();
  }
}

template <int DT, int M, int DS>
struct RunTables {
  static hipError_t run(const unsigned char* q, uint64_t nq, const float* cb,
                        float* out, hipStream_t s) {
    uint32_t grid = (uint32_t)(nq < 4096 ? nq : 4096);
    hipLaunchKernelGGL((table_kernel<DT, M, DS>), dim3(grid), dim3(256), 0, s,
                       q, nq, cb, out);
    return hipGetLastError();
  }
};

template <int DT, int M, int DS>
struct RunRerank {
  static hipError_t run(const DeviceIndex& ix, const unsigned char* q,
                        uint64_t nq, const uint32_t* cand, uint32_t c_max,
                        uint32_t k, uint32_t* ids, float* d, hipStream_t s) {
    uint32_t P = pow2ceil(c_max);
    size_t lds = (size_t)(P > k ? P : pow2ceil(k)) * 8;
    uint32_t grid = (uint32_t)(nq < 8192 ? nq : 8192);
    hipLaunchKernelGGL((rerank_kernel<DT, M * DS>), dim3(grid), dim3(kWave),
                       lds, s, ix.base, ix.n, q, nq, cand, c_max, k, ids, d);
    return hipGetLastError();
  }
};

// splitmix64 (Steele, Lea and Flood; the finaliser of Vigna's generator):
// a counter-based source of uniform 64-bit values.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t fold(uint4 v) {
  return v.x ^ v.y ^ v.z ^ v.w;
}
__device__ __forceinline__ uint32_t fold(uint32_t v) { return v; }

// Reads nreads random rows of `words` W-words (row r at src + r * stride):
// one wave per row, every lane a word (up to 8 words per lane).  The xor of
// the data decides a store that practically never happens, which keeps
// every load.
template <typename W>
__global__ __launch_bounds__(256) void probe_kernel(
    const unsigned char* __restrict__ src, uint64_t rows, uint32_t stride,
    uint32_t words, uint64_t nreads, uint64_t seed, uint64_t* sink) {
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) /
                        kWave;
  const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / kWave;
  uint32_t acc = 0;
  for (uint64_t i = wave; i < nreads; i += nw) {
    const uint64_t r = splitmix64(seed + i) % rows;
    const W* p = reinterpret_cast<const W*>(src + r * stride);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const uint32_t c = lane + (uint32_t)t * kWave;
      if (c < words) acc ^= fold(p[c]);
    }
  }
  if (acc == 0x2545F491u) sink[0] = wave;
}

// FP32 to bfloat16, to the nearest with ties to the even significand:
// adding 0x7FFF plus the lowest kept bit carries into the kept bits exactly
// when the dropped half is above the midpoint, or at it with an odd kept
// part.  Finite inputs (the base is finite data).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t b = __float_as_uint(x);
  return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// The PQ table with BF16 MFMA and FP32 accumulation (the precision form's
// table build): T[q][j][c] = |q_j|^2 + |c|^2 - 2 <bf16(q_j), bf16(c)>,
// the norms summed in FP32 from the unrounded coordinates, in order.  One
// wave per tile of 32 queries: for each subspace, v_mfma_f32_32x32x4_2b_bf16
// multiplies the 32 queries (rows, K = 4 coordinates per block) by 64
// centroids (block b holds 32 of them), so four MFMAs cover the 256
// centroids of a subspace of d/m = 4; d/m = 2 pads K with zeros, d/m = 8
// takes two K chunks; each wave covers kMfmaJ subspaces.  Lane layout
// (gfx950): A and B lane l feed block
// l / 32, row or column l % 32; result register v of lane l is block
// v / 16, row 8 ((v % 16) / 4) + 4 (l / 32) + v % 4, column l % 32.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x32_t __attribute__((ext_vector_type(32)));

constexpr int kMfmaJ = 8;  // subspaces per wave (grid y = m / kMfmaJ)

template <int DT, int M, int DS>
__global__ __launch_bounds__(64) void table_mfma_kernel(
    const unsigned char* __restrict__ queries, uint64_t nq,
    const float* __restrict__ cb, float* __restrict__ out) {
  constexpr int D = M * DS;
  constexpr int KC = (DS + 3) / 4;  // K chunks of 4 coordinates
  static_assert(M % kMfmaJ == 0, "subspaces are taken kMfmaJ at a time");
  __shared__ float qn_s[kMfmaJ][32];  // |q_j|^2 of the tile's 32 queries
  const int lane = threadIdx.x;
  const int half = lane >> 5, i = lane & 31;
  const uint64_t q0 = (uint64_t)blockIdx.x * 32;
  const int j0 = blockIdx.y * kMfmaJ;
  // this lane's query row (rows past nq read query q0, and are not written)
  const uint64_t qa = q0 + i < nq ? q0 + i : q0;
  const unsigned char* q = queries + qa * D * Elem<DT>::size;
  if (half == 0) {
    for (int jj = 0; jj < kMfmaJ; ++jj) {
      float s = 0.0f;
#pragma unroll
      for (int t = 0; t < DS; ++t) {
        const float v = Elem<DT>::f(q, (j0 + jj) * DS + t);
        s = s + v * v;
      }
      qn_s[jj][i] = s;
    }
  }
  __syncthreads();
  for (int j = j0; j < j0 + kMfmaJ; ++j) {
    bf16x4_t a[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t = kc * 4 + k;
        a[kc][k] = t < DS ? (short)to_bf16(Elem<DT>::f(q, j * DS + t)) : 0;
      }
    float qn[16];  // |q_j|^2 of the rows this lane's results belong to
#pragma unroll
    for (int v = 0; v < 16; ++v)
      qn[v] = qn_s[j - j0][8 * (v / 4) + 4 * half + v % 4];
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      const int cb0 = 64 * c4;
      const float* cen = cb + ((size_t)j * 256 + cb0 + 32 * half + i) * DS;
      bf16x4_t b[KC];
      float cn = 0.0f;
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int t = kc * 4 + k;
          const float v = t < DS ? cen[t] : 0.0f;
          b[kc][k] = (short)to_bf16(v);
          if (t < DS) cn = cn + v * v;
        }
      // |c|^2 of block 0's and block 1's column of this lane
      const float cn_other = __shfl_xor(cn, 32);
      const float cnb[2] = {half == 0 ? cn : cn_other,
                            half == 0 ? cn_other : cn};
      f32x32_t acc = {};
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
        acc = __builtin_amdgcn_mfma_f32_32x32x4bf16_1k(a[kc], b[kc], acc, 0,
                                                       0, 0);
#pragma unroll
      for (int v = 0; v < 32; ++v) {
        const int blk = v / 16, vv = v % 16;
        const uint64_t row = q0 + 8 * (vv / 4) + 4 * half + vv % 4;
        if (row < nq) {
          const float tq = qn[vv] + cnb[blk];
          out[row * (uint64_t)M * 256 + (uint64_t)j * 256 + cb0 + 32 * blk +
              i] = tq - 2.0f * acc[v];
        }
      }
    }
  }
}

template <int DT, int M, int DS>
struct RunTablesMfma {
  static hipError_t run(const unsigned char* q, uint64_t nq, const float* cb,
                        float* out, hipStream_t s) {
    const uint64_t grid = (nq + 31) / 32;
    if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((table_mfma_kernel<DT, M, DS>),
                       dim3((uint32_t)grid, M / kMfmaJ), dim3(64), 0, s, q, nq,
                       cb, out);
    return hipGetLastError();
  }
};

__global__ __launch_bounds__(256) void bf16_base_kernel(
    const float* __restrict__ base, uint64_t total,
    uint16_t* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
       i < total; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = to_bf16(base[i]);
}

// Sum of squares of each bfloat16 row, coordinates in order, FP32.
__global__ __launch_bounds__(256) void bf16_norm_kernel(
    const uint16_t* __restrict__ b16, uint64_t n, uint32_t d,
    float* __restrict__ norms) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (uint64_t)gridDim.x * blockDim.x) {
    const uint16_t* x = b16 + r * d;
    float acc = 0.0f;
    for (uint32_t t = 0; t < d; ++t) {
      const float v = __uint_as_float((uint32_t)x[t] << 16);
      const float sq = v * v;
      acc = acc + sq;
    }
    norms[r] = acc;
  }
}

}  // namespace

hipError_t launch_bf16_base(const float* base, uint64_t n, uint32_t d,
                            uint16_t* out16, float* norms, hipStream_t s) {
  const uint64_t total = n * d;
  const uint32_t g1 =
      (uint32_t)std::min<uint64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(bf16_base_kernel, dim3(g1), dim3(256), 0, s, base, total,
                     out16);
  const uint32_t g2 = (uint32_t)std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(bf16_norm_kernel, dim3(g2), dim3(256), 0, s, out16, n, d,
                     norms);
  return hipGetLastError();
}

uint32_t pow2ceil(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

bool supported(int dtype, uint32_t m, uint32_t ds) {
  if (dtype < kF32 || dtype > kI8) return false;
#define BANG_OK_SHAPE(MM, DD) \
  if (m == MM && ds == DD) return true;
  BANG_SHAPES(BANG_OK_SHAPE)
#undef BANG_OK_SHAPE
  return false;
}

static uint32_t lblock_for(uint32_t L) {
  const uint32_t b = (L + kWave - 1) / kWave;
  return b < (uint32_t)kPer ? b : (uint32_t)kPer;
}

static uint32_t lrow_for(uint32_t L) {
  const uint32_t sup = kWave * lblock_for(L);
  return (L + sup - 1) / sup * sup;
}

static size_t table_entry_bytes(int table) {
  return table == kTabF32 ? 4 : (table == kTabF16 ? 2 : 1);
}

// Table region: the table (plus the u8 form's m offsets).  After the search
// the re-rank sorts its keys in this region and the worklist buffer behind
// it when they fit (else it selects in global memory).
static size_t region0_bytes(uint32_t m, int tab) {
  if (tab == kTabExact) return 0;  // no table, no re-rank keys
  const size_t table = (size_t)m * 256 * table_entry_bytes(tab) +
                       (tab == kTabU8 ? (size_t)m * 4 : 0);
  return (table + 15) / 16 * 16;
}

size_t search_lds_bytes(uint32_t m, uint32_t L, uint32_t iter_cap,
                        int table) {
  (void)iter_cap;
  const size_t lrow = lrow_for(L);
  const size_t hist = (lrow + 4 + 15) / 16 * 16;
  return region0_bytes(m, table) + lrow * 8 + (kWave + 4) * 8 + hist;
}

uint32_t row_ids_bytes(uint32_t R) { return (4 * R + 15) / 16 * 16; }

uint32_t row_stride_bytes(uint32_t R, uint32_t m) {
  return (row_ids_bytes(R) + R * m + 15) / 16 * 16;
}

hipError_t launch_pack(const uint32_t* adj, const uint8_t* codes, uint32_t n,
                       uint32_t R, uint32_t m, unsigned char* rows,
                       hipStream_t s) {
  const uint64_t total = (uint64_t)n * R;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(pack_rows_kernel, dim3(grid), dim3(256), 0, s, adj, codes,
                     n, R, m, row_ids_bytes(R), row_stride_bytes(R, m), rows);
  return hipGetLastError();
}

uint32_t seen_words_for(uint32_t n) { return (n + 1023u) / 1024u * 32u; }

uint32_t seen_log_entries() { return kSeenLog; }

// Variant number of a search: host-resident adjacency (bit 0) | filter << 1
// | timed << 3 (search_variants.hip).
static int variant_of(bool host, int filter, bool phases) {
  return (host ? 1 : 0) | (filter << 1) | (phases ? 8 : 0);
}

hipError_t search_occupancy(const DeviceIndex& ix, int table, int filter,
                            bool phases, size_t lds, int* per_cu) {
  const int dt = ix.dtype;
  const uint32_t m = ix.m, ds = ix.d / ix.m;
  switch (variant_of(ix.hadj != nullptr, filter, phases)) {
    case 0: return search_occupancy_v0(dt, m, ds, table, lds, per_cu);
    case 1: return search_occupancy_v1(dt, m, ds, table, lds, per_cu);
    case 2: return search_occupancy_v2(dt, m, ds, table, lds, per_cu);
    case 3: return search_occupancy_v3(dt, m, ds, table, lds, per_cu);
    case 4: return search_occupancy_v4(dt, m, ds, table, lds, per_cu);
    case 5: return search_occupancy_v5(dt, m, ds, table, lds, per_cu);
    case 8: return search_occupancy_v8(dt, m, ds, table, lds, per_cu);
    case 12: return search_occupancy_v12(dt, m, ds, table, lds, per_cu);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tables(const DeviceIndex& ix, const void* queries,
                         uint64_t nq, float* out, hipStream_t s) {
  return dispatch<RunTables>(ix.dtype, ix.m, ix.d / ix.m,
                             (const unsigned char*)queries, nq, ix.cb, out, s);
}

hipError_t launch_tables_mfma(const DeviceIndex& ix, const void* queries,
                              uint64_t nq, float* out, hipStream_t s) {
  return dispatch<RunTablesMfma>(ix.dtype, ix.m, ix.d / ix.m,
                                 (const unsigned char*)queries, nq, ix.cb, out,
                                 s);
}

hipError_t launch_search(const DeviceIndex& ix, const SearchLaunch& l,
                         hipStream_t s) {
  const size_t lds0 = search_lds_bytes(ix.m, l.L, l.iter_cap, l.table);
  if (l.cache_slots &&
      (l.table != kTabExact || l.bloom || l.seen || l.cache_slots < 256 ||
       (l.cache_slots & (l.cache_slots - 1))))
    return hipErrorInvalidValue;
  const size_t lds = lds0 + 4 * (size_t)l.cache_slots;
  SearchArgs a;
  a.base = ix.base;
  a.rows = ix.rows;
  a.hadj = ix.hadj;
  a.codes = ix.codes;
  a.cb = ix.cb;
  a.queries = (const unsigned char*)l.queries;
  a.nq = l.nq;
  a.n = ix.n;
  a.R = ix.R;
  a.medoid = ix.medoid;
  a.row_stride = row_stride_bytes(ix.R, ix.m);
  a.row_ids = row_ids_bytes(ix.R);
  a.k = l.k;
  a.Lcap = l.L;
  a.c_max = l.c_max;
  a.iter_cap = l.iter_cap;
  a.lblock = lblock_for(l.L);
  a.lrow = lrow_for(l.L);
  a.region0 = (uint32_t)region0_bytes(ix.m, l.table);
  a.s_cap = (l.flags & 1u) ? 0u : (a.region0 + 8u * a.lrow) / 8u;
  a.out_ids = l.out_ids;
  a.out_dists = l.out_dists;
  a.qL = l.qL;
  a.qk = l.qk;
  a.out_cand = l.out_cand;
  a.cand_stride = l.cand_stride;
  a.out_counters = l.out_counters;
  a.out_times = l.out_times;
  a.out_phases = l.out_phases;
  a.cscratch = l.cscratch;
  a.bloom = l.bloom;
  a.bloom_epoch = l.bloom_epoch;
  a.abort_flag = l.abort_flag;
  a.abort_fired = l.abort_fired;
  a.base16 = l.rerank_bf16 ? ix.base16 : nullptr;
  a.norm16 = l.rerank_bf16 ? ix.norm16 : nullptr;
  a.tables = l.tables;
  a.order = l.order;
  a.seen = l.seen;
  a.seen_log = l.seen_log;
  a.seen_words = l.seen_words;
  a.seen_cap = std::min(l.seen_cap, kSeenLog);
  a.cache_off = (uint32_t)lds0;
  a.cache_slots = l.cache_slots;
  // slot = the top log2(cache_slots) bits of the 32-bit product
  a.cache_shift =
      l.cache_slots ? 32u - (uint32_t)__builtin_ctz(l.cache_slots) : 0u;
  a.qcounter = l.qcounter;
  const int dt = ix.dtype;
  const uint32_t m = ix.m, ds = ix.d / ix.m;
  const int filter =
      a.bloom ? kFilterBloom : (a.seen ? kFilterSeen : kFilterUnion);
  if (a.seen && (!a.seen_log || a.seen_words < seen_words_for(ix.n)))
    return hipErrorInvalidValue;
  switch (variant_of(a.hadj != nullptr, filter, a.out_phases != nullptr)) {
    case 0: return search_launch_v0(a, dt, m, ds, l.table, l.grid, lds, s);
    case 1: return search_launch_v1(a, dt, m, ds, l.table, l.grid, lds, s);
    case 2: return search_launch_v2(a, dt, m, ds, l.table, l.grid, lds, s);
    case 3: return search_launch_v3(a, dt, m, ds, l.table, l.grid, lds, s);
    case 4: return search_launch_v4(a, dt, m, ds, l.table, l.grid, lds, s);
    case 5: return search_launch_v5(a, dt, m, ds, l.table, l.grid, lds, s);
    case 8: return search_launch_v8(a, dt, m, ds, l.table, l.grid, lds, s);
    case 12: return search_launch_v12(a, dt, m, ds, l.table, l.grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_probe(const DeviceIndex& ix, uint64_t nreads, uint64_t seed,
                        uint64_t* sink, uint32_t grid, uint32_t* row_bytes,
                        hipStream_t s) {
  if (ix.hadj) {
    // the R ids of a row, as load_row reads them across the host link
    *row_bytes = 4 * ix.R;
    if (nreads == 0) return hipSuccess;
    hipLaunchKernelGGL(probe_kernel<uint32_t>, dim3(grid), dim3(256), 0, s,
                       reinterpret_cast<const unsigned char*>(ix.hadj),
                       (uint64_t)ix.n, 4 * ix.R, ix.R, nreads, seed, sink);
  } else {
    const uint32_t bytes = (row_ids_bytes(ix.R) + ix.R * ix.m + 15) / 16 * 16;
    *row_bytes = bytes;
    if (nreads == 0) return hipSuccess;
    hipLaunchKernelGGL(probe_kernel<uint4>, dim3(grid), dim3(256), 0, s,
                       ix.rows, (uint64_t)ix.n, row_stride_bytes(ix.R, ix.m),
                       bytes / 16, nreads, seed, sink);
  }
  return hipGetLastError();
}

hipError_t launch_rerank(const DeviceIndex& ix, const void* queries,
                         uint64_t nq, const uint32_t* cand, uint32_t c_max,
                         uint32_t k, uint32_t* out_ids, float* out_dists,
                         hipStream_t s) {
  return dispatch<RunRerank>(ix.dtype, ix.m, ix.d / ix.m, ix,
                             (const unsigned char*)queries, nq, cand, c_max, k,
                             out_ids, out_dists, s);
}

}  // namespace bang
