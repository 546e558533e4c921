// The batched greedy search of one query per wavefront (gfx950, MI355X):
// device helpers and the search kernel template.  bang_kernels.hip (table,
// re-rank and row-packing kernels, host side) and search_variants.hip (one
// translation unit per search variant) include it.
//
// Per query, one wave of 64 lanes in a persistent workgroup:
//  * builds the query's PQ table into LDS (section "Construction of
//    PQDistTable in Parallel": centroids across lanes, subspaces in order);
//  * expands the first unvisited worklist entry u*: lane r holds slot r of
//    u*'s packed adjacency row (ids and the neighbours' codes, one
//    coalesced load) and sums its neighbour's m table entries in subspace
//    order (section "Parallel Neighbour Distance Computation");
//  * ranks each new key in the sorted LDS worklist (radix-4 search; equal
//    node = already present, dropped: Algorithm 1's set union) and merges
//    the live keys in place (position = own index + rank in the other
//    list, section "Parallel Merge"), keeping the first t;
//  * picks the next node before the merge from the two candidates of the
//    eager rule and requests its row at once (section "Prefetching
//    Candidate Nodes"), so the load overlaps the merge;
//  * re-ranks the expanded nodes with exact distances (section
//    "Re-ranking").
//
// Keys: (float bits of the distance) << 32 | id << 1 | visited.  Distances
// are non-negative, so unsigned key order is (distance, id) order; ids are
// unique in a worklist, so the visited bit never decides an order.
//
// All floating point here is FP32 with contraction off and a fixed order,
// which makes results bit-identical to a sequential reference.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "internal.h"

#pragma clang fp contract(off)

namespace bang {

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kInf = ~0ull;
constexpr int kWave = 64;
// s_waitcnt immediate for vmcnt(0) alone (gfx9 encoding: expcnt and lgkmcnt
// at their maxima, no wait on them)
constexpr unsigned kWaitVmem0 = 0x0F70;

__device__ __forceinline__ uint64_t make_key(float d, uint32_t id) {
  return ((uint64_t)__float_as_uint(d) << 32) | ((uint64_t)id << 1);
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) {
  return ((uint32_t)k) >> 1;
}
__device__ __forceinline__ float key_dist(uint64_t k) {
  return __uint_as_float((uint32_t)(k >> 32));
}

template <int DT>
struct Elem;
template <>
struct Elem<kF32> {
  static constexpr int size = 4;
  __device__ static float f(const unsigned char* p, int i) {
    return reinterpret_cast<const float*>(p)[i];
  }
};
template <>
struct Elem<kU8> {
  static constexpr int size = 1;
  __device__ static float f(const unsigned char* p, int i) {
    return (float)p[i];
  }
};
template <>
struct Elem<kI8> {
  static constexpr int size = 1;
  __device__ static float f(const unsigned char* p, int i) {
    return (float)(int8_t)p[i];
  }
};

// One centroid's DS coordinates (16-, 8- or 4-byte loads).
template <int DS>
__device__ __forceinline__ void load_centroid(const float* __restrict__ cent,
                                              float (&cv)[DS]) {
  if constexpr (DS % 4 == 0) {
#pragma unroll
    for (int t = 0; t < DS; t += 4) {
      float4 v = *reinterpret_cast<const float4*>(cent + t);
      cv[t] = v.x; cv[t + 1] = v.y; cv[t + 2] = v.z; cv[t + 3] = v.w;
    }
  } else if constexpr (DS % 2 == 0) {
#pragma unroll
    for (int t = 0; t < DS; t += 2) {
      float2 v = *reinterpret_cast<const float2*>(cent + t);
      cv[t] = v.x; cv[t + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < DS; ++t) cv[t] = cent[t];
  }
}

// One table entry: sum over the subvector in coordinate order, FP32.
template <int DS>
__device__ __forceinline__ float entry_sum(const float* qv,
                                           const float (&cv)[DS]) {
  float acc = 0.0f;
#pragma unroll
  for (int t = 0; t < DS; ++t) {
    float diff = qv[t] - cv[t];
    float sq = diff * diff;
    acc = acc + sq;
  }
  return acc;
}

template <int DS>
__device__ __forceinline__ float table_entry(const float* qv,
                                             const float* __restrict__ cent) {
  float cv[DS];
  load_centroid<DS>(cent, cv);
  return entry_sum<DS>(qv, cv);
}

// Table of one query: T[j*256 + c], `nthr` threads starting at `tid`.
template <int DT, int M, int DS>
__device__ __forceinline__ void build_table(const unsigned char* q,
                                            const float* __restrict__ cb,
                                            float* T, int tid, int nthr) {
  for (int j = 0; j < M; ++j) {
    float qv[DS];
#pragma unroll
    for (int t = 0; t < DS; ++t) qv[t] = Elem<DT>::f(q, j * DS + t);
    for (int c = tid; c < 256; c += nthr)
      T[j * 256 + c] = table_entry<DS>(qv, cb + ((size_t)j * 256 + c) * DS);
  }
}

// ADC of one compressed vector: sum of m table entries, subspace order.
template <int M>
__device__ __forceinline__ float adc(const float* T,
                                     const uint8_t* __restrict__ code) {
  static_assert(M % 16 == 0, "codes are gathered 16 bytes at a time");
  uint4 v[M / 16];
#pragma unroll
  for (int c = 0; c < M / 16; ++c)
    v[c] = *reinterpret_cast<const uint4*>(code + 16 * c);
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < M / 16; ++c) {
    const uint32_t w[4] = {v[c].x, v[c].y, v[c].z, v[c].w};
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      uint32_t byte = (w[b >> 2] >> (8 * (b & 3))) & 0xFFu;
      acc = acc + T[(16 * c + b) * 256 + byte];
    }
  }
  return acc;
}

// Table storage of the search: canonical FP32, or the precision form's
// half (times a power-of-two scale) or u8 (per-subspace offset, one scale).
// Both reduced forms are derived from the canonical FP32 entries, so they
// are as deterministic as the FP32 table itself.  kTabExact: no table; the
// search ranks by exact distances and skips the re-rank (the paper's
// Exact-distance Version, section "Implementation Variants").
enum TableKind : int { kTabF32 = 0, kTabF16 = 1, kTabU8 = 2, kTabExact = 3 };

template <int TT>
struct Tab;
template <>
struct Tab<kTabF32> {
  using E = float;
};
template <>
struct Tab<kTabF16> {
  using E = uint16_t;
};
template <>
struct Tab<kTabU8> {
  using E = uint8_t;
};
template <>
struct Tab<kTabExact> {
  using E = uint8_t;  // no table
};
template <int TT>
constexpr int table_bytes(int M) {
  return TT == kTabExact ? 0 : M * 256 * (int)sizeof(typename Tab<TT>::E);
}

__device__ __forceinline__ float f16_bits_to_f32(uint16_t h) {
  return (float)__builtin_bit_cast(_Float16, h);
}

// Maximum / minimum of one float per lane across the wave (DPP), returned
// to every lane.  `ident` is the identity for lanes outside a row.
template <bool MAX>
__device__ __forceinline__ float wave_minmax(float v, float ident) {
  const uint32_t id = __float_as_uint(ident);
#define BANG_MM(CTRL, RM)                                                    \
  {                                                                          \
    float t = __uint_as_float((uint32_t)__builtin_amdgcn_update_dpp(         \
        (int)id, (int)__float_as_uint(v), CTRL, RM, 0xF, false));            \
    v = MAX ? (t > v ? t : v) : (t < v ? t : v);                             \
  }
  BANG_MM(0x111, 0xF) BANG_MM(0x112, 0xF) BANG_MM(0x114, 0xF)
  BANG_MM(0x118, 0xF) BANG_MM(0x142, 0xA) BANG_MM(0x143, 0xC)
#undef BANG_MM
  return __uint_as_float(
      __builtin_amdgcn_readlane(__float_as_uint(v), 63));
}

// The query vector spread over one wave for the table build: lane l holds
// bytes [4l, 4l + 4) of each 256-byte block, so that every coordinate is one
// cross-lane read away instead of a memory round trip per subspace.
template <int DT, int D>
struct QueryLanes {
  static constexpr int kBytes = D * Elem<DT>::size;
  static constexpr int kRegs = (kBytes + 4 * kWave - 1) / (4 * kWave);
  static_assert(kBytes % 4 == 0, "the query is read in 4-byte words");
  uint32_t w[kRegs];

  __device__ __forceinline__ void load(const unsigned char* q, int lane) {
    const uint32_t* q4 = reinterpret_cast<const uint32_t*>(q);
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
      const int wi = lane + kWave * r;
      w[r] = wi * 4 < kBytes ? q4[wi] : 0u;
    }
  }
  // coordinate i (the same i on every lane), converted as Elem<DT>::f does
  __device__ __forceinline__ float elem(int i) const {
    const int b = i * Elem<DT>::size;
    const int wi = b >> 2;
    uint32_t v = w[0];
#pragma unroll
    for (int r = 1; r < kRegs; ++r) v = (wi >> 6) == r ? w[r] : v;
    v = (uint32_t)__builtin_amdgcn_readlane((int)v, wi & (kWave - 1));
    if constexpr (DT == kF32) {
      return __uint_as_float(v);
    } else if constexpr (DT == kU8) {
      return (float)((v >> (8 * (b & 3))) & 0xFFu);
    } else {
      return (float)(int8_t)(v >> (8 * (b & 3)));
    }
  }
};

// This lane's entries of the query's table, subspace by subspace: f(j, e)
// receives the entries of centroids lane + 64 r (r = 0..3) of subspace j.
// Centroids are loaded JU subspaces (16 floats a lane, or one subspace) at a
// time into two buffers: the loads of the next block are in flight while
// one is scored, so the build waits about M / JU memory latencies, not 4 M
// (d/m >= 8: one buffer of one subspace).
template <int DT, int M, int DS, class F>
__device__ __forceinline__ void table_entries(
    const QueryLanes<DT, M * DS>& Q, const float* __restrict__ cb, int lane,
    F&& f) {
  constexpr int R = 256 / kWave;
  constexpr int JU = DS >= 4 ? 1 : 4 / DS;
  static_assert(M % (2 * JU) == 0, "subspaces are taken 2 JU at a time");
  auto load = [&](float (&cv)[JU][R][DS], int j0) {
#pragma unroll
    for (int jj = 0; jj < JU; ++jj)
#pragma unroll
      for (int r = 0; r < R; ++r)
        load_centroid<DS>(
            cb + ((size_t)(j0 + jj) * 256 + lane + kWave * r) * DS, cv[jj][r]);
  };
  auto score = [&](const float (&cv)[JU][R][DS], int j0) {
#pragma unroll
    for (int jj = 0; jj < JU; ++jj) {
      float qv[DS];
#pragma unroll
      for (int t = 0; t < DS; ++t) qv[t] = Q.elem((j0 + jj) * DS + t);
      float e[R];
#pragma unroll
      for (int r = 0; r < R; ++r) e[r] = entry_sum<DS>(qv, cv[jj][r]);
      f(j0 + jj, e);
    }
  };
  float ca[JU][R][DS], cbuf[JU][R][DS];
  if constexpr (DS >= 8) {
    // a subspace alone fills 32 registers a lane: one buffer, so that the
    // build does not raise the register count (and cut occupancy) of the
    // search that calls it
#pragma unroll 1
    for (int j0 = 0; j0 < M; j0 += JU) {
      load(ca, j0);
      score(ca, j0);
    }
    return;
  }
  load(ca, 0);
#pragma unroll 1
  for (int j0 = 0; j0 < M; j0 += 2 * JU) {
    load(cbuf, j0 + JU);
    score(ca, j0);
    // past the last block the first one is loaded again (unused): the loads
    // stay unconditional, so the wait for cbuf does not include them
    load(ca, j0 + 2 * JU < M ? j0 + 2 * JU : 0);
    score(cbuf, j0 + JU);
  }
}

// The same entries read from a table built beforehand (Tq: [m][256] FP32).
template <int M, class F>
__device__ __forceinline__ void table_entries_given(const float* __restrict__ Tq,
                                                    int lane, F&& f) {
  constexpr int R = 256 / kWave;
#pragma unroll 4
  for (int j = 0; j < M; ++j) {
    float e[R];
#pragma unroll
    for (int r = 0; r < R; ++r) e[r] = Tq[j * 256 + lane + kWave * r];
    f(j, e);
  }
}

// The query's table in LDS, in the storage form TT (one wave, 64 lanes),
// built from the codebooks or, when Tq is not null, taken from the FP32
// table there.  lo (U8 only): m floats of LDS for the per-subspace offsets.
// Out of line: it runs once per query, and its registers are then not
// allocated together with the search loop's (measured 1-3% faster at
// L=768).
template <int DT, int M, int DS, int TT>
__device__ __attribute__((noinline)) void build_table_q(QueryLanes<DT, M * DS> Q,
                                              const float* __restrict__ cb,
                                              const float* __restrict__ Tq,
                                              void* Tv, float* lo, int lane) {
  constexpr int R = 256 / kWave;
  auto entries = [&](auto&& f) {
    if (Tq)
      table_entries_given<M>(Tq, lane, f);
    else
      table_entries<DT, M, DS>(Q, cb, lane, f);
  };
  if constexpr (TT == kTabF32) {
    float* T = reinterpret_cast<float*>(Tv);
    entries([&](int j, const float (&e)[R]) {
#pragma unroll
      for (int r = 0; r < R; ++r) T[j * 256 + lane + kWave * r] = e[r];
    });
  } else {
    // pass 1: the statistics the storage needs
    float mx = 0.0f;  // F16: largest entry; U8: widest subspace range
    entries([&](int j, const float (&e)[R]) {
      float vmin = __uint_as_float(0x7F800000u), vmax = 0.0f;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vmin = e[r] < vmin ? e[r] : vmin;
        vmax = e[r] > vmax ? e[r] : vmax;
      }
      if constexpr (TT == kTabF16) {
        mx = vmax > mx ? vmax : mx;
      } else {
        const float l = wave_minmax<false>(vmin, __uint_as_float(0x7F800000u));
        const float h = wave_minmax<true>(vmax, 0.0f);
        const float range = h - l;
        mx = range > mx ? range : mx;
        if (lane == 0) lo[j] = l;
      }
    });
    float mul;
    if constexpr (TT == kTabF16) {
      mx = wave_minmax<true>(mx, 0.0f);
      mul = 1.0f;
      while (mx * mul > 65504.0f) mul = mul * 0.5f;
    } else {
      mul = mx > 0.0f ? 255.0f / mx : 0.0f;
      __syncthreads();  // lo[] visible to every lane
    }
    // pass 2: the entries again (bit-identical), stored in the reduced form
    typename Tab<TT>::E* T = reinterpret_cast<typename Tab<TT>::E*>(Tv);
    entries([&](int j, const float (&e)[R]) {
      const float lj = (TT == kTabU8) ? lo[j] : 0.0f;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int c = lane + kWave * r;
        if constexpr (TT == kTabF16) {
          const float sv = e[r] * mul;
          T[j * 256 + c] = __builtin_bit_cast(uint16_t, (_Float16)sv);
        } else {
          const float diff = e[r] - lj;
          const float v = __builtin_rintf(diff * mul);
          T[j * 256 + c] = (uint8_t)(v > 255.0f ? 255.0f : v);
        }
      }
    });
  }
}

// ADC under storage TT: FP32 sum of the (widened) entries in subspace order;
// for U8 the exact integer sum, returned as FP32 (exact below 2^24).
// (byte B of w) << S in one instruction (SDWA byte select): the byte
// offset of entry `code` in a table row of 2^S-byte entries.
#define BANG_SDWA_SHL(S, B)                                               \
  asm("v_lshlrev_b32_sdwa %0, " #S ", %1 dst_sel:DWORD "                   \
      "dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_" #B             \
      : "=v"(r) : "v"(w))
template <int S, int B>
__device__ __forceinline__ uint32_t byte_shl(uint32_t w) {
  static_assert(S >= 0 && S <= 2 && B >= 0 && B <= 3, "byte_shl");
  if constexpr (S == 0) {
    return (w >> (8 * B)) & 0xFFu;
  } else {
    uint32_t r;
    if constexpr (S == 1 && B == 0) BANG_SDWA_SHL(1, 0);
    else if constexpr (S == 1 && B == 1) BANG_SDWA_SHL(1, 1);
    else if constexpr (S == 1 && B == 2) BANG_SDWA_SHL(1, 2);
    else if constexpr (S == 1 && B == 3) BANG_SDWA_SHL(1, 3);
    else if constexpr (B == 0) BANG_SDWA_SHL(2, 0);
    else if constexpr (B == 1) BANG_SDWA_SHL(2, 1);
    else if constexpr (B == 2) BANG_SDWA_SHL(2, 2);
    else BANG_SDWA_SHL(2, 3);
    return r;
  }
}
#undef BANG_SDWA_SHL

// ADC of one neighbour from its m codes (16 per uint4) against the query's
// table, which must start at LDS address 0: the search kernel puts it first
// in its dynamic LDS block and declares no static LDS.
template <int M, int TT>
__device__ __forceinline__ float adc_codes(const uint4 (&v)[M / 16]) {
  using E = typename Tab<TT>::E;
  // all M lookups are issued before the first add, so their LDS latencies
  // overlap; the adds then run in subspace order
  E e[M];
#pragma unroll
  for (int c = 0; c < M / 16; ++c) {
    const uint32_t w[4] = {v[c].x, v[c].y, v[c].z, v[c].w};
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      // entry (j, code) at byte offset (j*256 + code) * sizeof(E); the
      // byte offset of the code comes from one SDWA instruction, and the
      // table, the first thing in the dynamic LDS block, starts at LDS
      // address 0 (search_kernel declares no static LDS), so no base is
      // added
      constexpr int S = sizeof(E) == 4 ? 2 : (sizeof(E) == 2 ? 1 : 0);
      uint32_t off;
      switch (b & 3) {
        case 0: off = byte_shl<S, 0>(w[b >> 2]); break;
        case 1: off = byte_shl<S, 1>(w[b >> 2]); break;
        case 2: off = byte_shl<S, 2>(w[b >> 2]); break;
        default: off = byte_shl<S, 3>(w[b >> 2]); break;
      }
      using lds_E = __attribute__((address_space(3))) const E;
      e[16 * c + b] = *(reinterpret_cast<lds_E*>(static_cast<uintptr_t>(off)) +
                        (16 * c + b) * 256);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  float acc = 0.0f;
  uint32_t iacc = 0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    if constexpr (TT == kTabF32) acc = acc + e[j];
    else if constexpr (TT == kTabF16) acc = acc + f16_bits_to_f32(e[j]);
    else iacc += e[j];
  }
  return TT == kTabU8 ? (float)iacc : acc;
}

// Sum of the squares of the query's coordinates, integer data only (0 for
// FP32): the constant term of exact_dist.
template <int DT, int D>
__device__ __forceinline__ int32_t query_sq(const unsigned char* q) {
  if constexpr (DT == kF32) {
    return 0;
  } else {
    const uint32_t* qw = reinterpret_cast<const uint32_t*>(q);
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < D / 4; ++i) {
      if constexpr (DT == kU8)
        s = __builtin_amdgcn_udot4(qw[i], qw[i], s, false);
      else
        s = (uint32_t)__builtin_amdgcn_sdot4((int)qw[i], (int)qw[i], (int)s,
                                             false);
    }
    return (int32_t)s;
  }
}

// Exact squared distance between base row `id` and the query.  FP32 data:
// the differences squared and added left to right over the d coordinates.
// Integer data: sum (x - q)^2 = sum x^2 - 2 sum x q + qq (qq = query_sq),
// each sum exact from four-byte dot products, so the value is the plain
// integer sum (below 2^24, exact in FP32).
// EAGER: every load of the row is issued before the first product (one
// memory round trip, D/4 more registers); otherwise two chunks at a time.
// Float data: the row is read eight (EAGER) or four 16-byte chunks at a time.
template <int DT, int D, bool EAGER = false>
__device__ __forceinline__ float exact_dist(const void* __restrict__ base,
                                            uint32_t id,
                                            const unsigned char* q,
                                            int32_t qq) {
  if constexpr (DT == kF32) {
    const float4* x =
        reinterpret_cast<const float4*>((const float*)base + (size_t)id * D);
    const float* qq = reinterpret_cast<const float*>(q);
    float acc = 0.0f;
    // EAGER: eight 16-byte loads in flight instead of four
    constexpr int kUnroll = EAGER ? 8 : 4;
#pragma unroll kUnroll
    for (int c = 0; c < D / 4; ++c) {
      float4 v = x[c];
      const float xv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float diff = xv[t] - qq[4 * c + t];
        float sq = diff * diff;
        acc = acc + sq;
      }
    }
    return acc;
  } else {
    static_assert(D % 16 == 0, "rows are read 16 bytes at a time");
    const uint4* x = reinterpret_cast<const uint4*>(
        (const uint8_t*)base + (size_t)id * D);
    const uint32_t* qw = reinterpret_cast<const uint32_t*>(q);
    uint32_t xx = 0, xq = 0;
    uint4 row[EAGER ? D / 16 : 1];
    if constexpr (EAGER) {
#pragma unroll
      for (int c = 0; c < D / 16; ++c) row[c] = x[c];
    }
    constexpr int kUnroll = EAGER ? D / 16 : 2;
#pragma unroll kUnroll
    for (int c = 0; c < D / 16; ++c) {
      const uint4 v = EAGER ? row[EAGER ? c : 0] : x[c];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if constexpr (DT == kU8) {
          xx = __builtin_amdgcn_udot4(w[t], w[t], xx, false);
          xq = __builtin_amdgcn_udot4(w[t], qw[4 * c + t], xq, false);
        } else {
          xx = (uint32_t)__builtin_amdgcn_sdot4((int)w[t], (int)w[t], (int)xx,
                                                false);
          xq = (uint32_t)__builtin_amdgcn_sdot4((int)w[t], (int)qw[4 * c + t],
                                                (int)xq, false);
        }
      }
    }
    return (float)(int32_t)(xx - 2u * xq + (uint32_t)qq);
  }
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return ((uint64_t)hi << 32) | lo;
}

// v of the lowest lane set in the wave-uniform mask (nonzero): a scalar
// read of one lane, no LDS round trip.
__device__ __forceinline__ uint32_t first_of(uint32_t v, uint64_t mask) {
  return __builtin_amdgcn_readlane(v, __builtin_ctzll(mask));
}

// Cross-lane helpers on DPP (data-parallel primitives; no LDS round trip).
// dpp_ctrl encodings of the GFX9 family: row_shr:n = 0x110 + n,
// row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL,
                                               ROW_MASK, 0xF, false);
}

// Exclusive prefix sum of one value per lane across the wave.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t x) {
  uint32_t v = x;
  v += dpp<0x111>(0u, v);  // row_shr:1
  v += dpp<0x112>(0u, v);  // row_shr:2
  v += dpp<0x114>(0u, v);  // row_shr:4
  v += dpp<0x118>(0u, v);  // row_shr:8
  v += dpp<0x142, 0xA>(0u, v);  // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xC>(0u, v);  // row_bcast:31 into rows 2 and 3
  return v - x;
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t min_dpp(uint64_t v) {
  const uint32_t lo = dpp<CTRL, ROW_MASK>(0xFFFFFFFFu, (uint32_t)v);
  const uint32_t hi = dpp<CTRL, ROW_MASK>(0xFFFFFFFFu, (uint32_t)(v >> 32));
  const uint64_t t = ((uint64_t)hi << 32) | lo;
  return t < v ? t : v;
}

// Minimum of one u32 per lane across the wave, returned to every lane.
__device__ __forceinline__ uint32_t wave_min32(uint32_t v) {
  v = min(v, dpp<0x111>(0xFFFFFFFFu, v));
  v = min(v, dpp<0x112>(0xFFFFFFFFu, v));
  v = min(v, dpp<0x114>(0xFFFFFFFFu, v));
  v = min(v, dpp<0x118>(0xFFFFFFFFu, v));
  v = min(v, dpp<0x142, 0xA>(0xFFFFFFFFu, v));
  v = min(v, dpp<0x143, 0xC>(0xFFFFFFFFu, v));
  return __builtin_amdgcn_readlane(v, 63);
}

// Minimum of one u64 per lane across the wave, returned to every lane.
__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
  v = min_dpp<0x111>(v);
  v = min_dpp<0x112>(v);
  v = min_dpp<0x114>(v);
  v = min_dpp<0x118>(v);
  v = min_dpp<0x142, 0xA>(v);
  v = min_dpp<0x143, 0xC>(v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// Exact distances of the wave's 64 neighbours (lane r: neighbour nb of lane
// r) for integer data, with the base rows read cooperatively: G lanes, one
// 16-byte chunk each, share a row, so one load instruction covers 64/G
// whole rows instead of 64 scattered pieces.  Each lane adds the dot
// products of its chunk (sum x^2 - 2 sum x q: exact integers), a DPP
// reduction leaves each row's total in the last lane of its group, and
// lane r collects neighbour r's.  Integer sums are exact in any order, so
// the value equals exact_dist's.  qc = this lane's query chunk (zero past
// the row), qq = query_sq.  Only lanes 0..nlive-1 may hold a neighbour
// (wave-uniform nlive).  Every lane must call it (cross-lane).
template <int DT, int D>
__device__ __forceinline__ float coop_dist(const void* __restrict__ base,
                                           uint32_t nb, const uint4& qc,
                                           int32_t qq, int lane,
                                           uint32_t nlive = kWave) {
  constexpr int CH = D / 16;
  static_assert(D % 16 == 0 && CH >= 1 && CH <= 8, "rows of 16..128 bytes");
  constexpr int G = CH <= 2 ? 2 : (CH <= 4 ? 4 : 8);  // lanes per row
  constexpr int RPI = kWave / G;                      // rows per load
  const int c = lane % G, g = lane / G;
  const int cc = c < CH ? c : CH - 1;  // in-row chunk (masked below)
  uint4 v[G];
  bool ok[G];
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const uint32_t id = __shfl(nb, t * RPI + g);
    ok[t] = id != kNone && c < CH;
    // the loads of the second half of the lanes' rows are not issued when
    // they hold no neighbour (one wave-uniform test; a finer one costs
    // registers)
    v[t] = make_uint4(0u, 0u, 0u, 0u);
    if (t < G / 2 || nlive > (uint32_t)(kWave / 2))
      v[t] = reinterpret_cast<const uint4*>(
          (const uint8_t*)base + (size_t)(id != kNone ? id : 0u) * D)[cc];
  }
  const uint32_t qw[4] = {qc.x, qc.y, qc.z, qc.w};
  uint32_t part[G];
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const uint32_t w[4] = {v[t].x, v[t].y, v[t].z, v[t].w};
    uint32_t xx = 0, xq = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if constexpr (DT == kU8) {
        xx = __builtin_amdgcn_udot4(w[u], w[u], xx, false);
        xq = __builtin_amdgcn_udot4(w[u], qw[u], xq, false);
      } else {
        xx = (uint32_t)__builtin_amdgcn_sdot4((int)w[u], (int)w[u], (int)xx,
                                              false);
        xq = (uint32_t)__builtin_amdgcn_sdot4((int)w[u], (int)qw[u], (int)xq,
                                              false);
      }
    }
    uint32_t s = ok[t] ? xx - 2u * xq : 0u;
    // group total into the group's last lane (groups lie inside DPP rows)
    s += dpp<0x111>(0u, s);                     // row_shr:1
    if constexpr (G >= 4) s += dpp<0x112>(0u, s);  // row_shr:2
    if constexpr (G >= 8) s += dpp<0x114>(0u, s);  // row_shr:4
    part[t] = s;
  }
  // neighbour r was row slot r % RPI of load t = r / RPI
  const int src = (lane % RPI) * G + (G - 1);
  uint32_t tot = 0;
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const uint32_t x = __shfl(part[t], src);
    if (lane / RPI == t) tot = x;
  }
  return (float)(int32_t)(tot + (uint32_t)qq);
}

// The u64 at LDS byte address b (the dynamic LDS block starts at address
// 0: search_kernel declares no static LDS).
__device__ __forceinline__ uint64_t lds_u64(uint32_t b) {
  using lds_t = __attribute__((address_space(3))) const uint64_t;
  return *reinterpret_cast<lds_t*>(static_cast<uintptr_t>(b));
}

// Number P of entries of the sorted LDS list A[0..len) whose key, visited
// bit ignored, is below x's (1 <= len <= 1024, last = A[len-1]), and in ge
// the entry A[P] (kInf when P = len); A is at LDS byte address base.
// (a >> 1) < (x >> 1) is tested as a < (x & ~1).  Radix-4 lifting: three
// independent probes per level, half the dependent LDS reads of a binary
// search (those of the first level, the same for every key, given in top),
// down to a last level that reads the four entries P can be (pos ..
// pos+3): the first of them not below x is A[P], so ge comes from that
// level alone.  Probes past A[len-2] are clamped to A[len-1] = last,
// which is known not to be below x (a clamp instead of a branch); probes
// are kept as byte addresses, so each is one add and one clamp.
__device__ __forceinline__ uint32_t rank_in(uint32_t base, uint32_t len,
                                            uint64_t last,
                                            const uint64_t (&top)[3],
                                            uint64_t x, uint64_t& ge) {
  const uint64_t xs = x & ~1ull;
  if (last < xs) {
    ge = kInf;
    return len;
  }
  const uint32_t lim = len - 1;  // the answer is at most lim
  const uint32_t la = base + 8u * lim;
  // the first level's probes were read by the caller (top: A[255], A[511],
  // A[767], clamped to A[lim], which is not below x)
  uint32_t pa = base;  // address of A[pos]
  if (lim >= 256)
    pa += 2048u * ((uint32_t)(top[0] < xs) + (uint32_t)(top[1] < xs) +
                   (uint32_t)(top[2] < xs));
  for (uint32_t s = 64; s > 1; s >>= 2) {
    if (s > lim) continue;
    const uint64_t v1 = lds_u64(min(pa + 8u * (s - 1), la));
    const uint64_t v2 = lds_u64(min(pa + 8u * (2 * s - 1), la));
    const uint64_t v3 = lds_u64(min(pa + 8u * (3 * s - 1), la));
    pa += 8u * s *
          ((uint32_t)(v1 < xs) + (uint32_t)(v2 < xs) + (uint32_t)(v3 < xs));
  }
  // P is in pos .. pos+3 (and at most lim, where A[lim] = last is not
  // below x)
  const uint64_t v0 = lds_u64(min(pa, la));
  const uint64_t v1 = lds_u64(min(pa + 8u, la));
  const uint64_t v2 = lds_u64(min(pa + 16u, la));
  const uint64_t v3 = lds_u64(min(pa + 24u, la));
  const bool p0 = v0 < xs, p1 = v1 < xs, p2 = v2 < xs;
  ge = !p0 ? v0 : (!p1 ? v1 : (!p2 ? v2 : v3));
  return (pa - base) / 8u + (uint32_t)p0 + (uint32_t)p1 + (uint32_t)p2;
}

// Ascending bitonic sort of S[0..P) in LDS by one wave (P a power of two).
__device__ void lds_sort(uint64_t* S, uint32_t P, int lane) {
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = lane; i < P / 2; i += kWave) {
        uint32_t lo = 2 * i - (i & (stride - 1));
        uint32_t hi = lo + stride;
        bool asc = (lo & size) == 0;
        uint64_t x = S[lo], y = S[hi];
        if ((x > y) == asc) {
          S[lo] = y;
          S[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ uint32_t pow2ceil_dev(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Sort the first `cnt` keys of S (padding to a power of two with +inf) and
// write the first k as (id, distance), padding with (NONE, +inf).
__device__ void sort_and_emit(uint64_t* S, uint32_t cnt, uint32_t k,
                              uint32_t* out_ids, float* out_d, int lane) {
  uint32_t P = pow2ceil_dev(cnt > 0 ? cnt : 1);
  for (uint32_t i = cnt + lane; i < P; i += kWave) S[i] = kInf;
  __syncthreads();
  lds_sort(S, P, lane);
  for (uint32_t i = lane; i < k; i += kWave) {
    uint64_t key = i < cnt ? S[i] : kInf;
    out_ids[i] = key == kInf ? kNone : key_id(key);
    out_d[i] = key == kInf ? __uint_as_float(0x7F800000u) : key_dist(key);
  }
}

// The k <= 64 smallest of the distinct keys S[i], i < cnt, ascending, to
// the outputs (padded with (NONE, +inf)).  Lane l holds in best/at the
// smallest of its own keys (i = l mod 64).  Each round the wave minimum is
// the next result; only the lane that owned it rescans its keys.  k rounds
// of a wave minimum instead of a sort of all cnt keys.
__device__ void select_and_emit(uint64_t* S, uint32_t cnt, uint32_t k,
                                uint64_t best, uint32_t at, uint32_t* out_ids,
                                float* out_d, int lane) {
  uint64_t mine = kInf;  // lane r: the r-th result
  for (uint32_t r = 0; r < k; ++r) {
    const uint64_t m = wave_min64(best);
    if ((uint32_t)lane == r) mine = m;
    if (m == kInf) break;
    if (best == m) {  // one lane: the keys are distinct
      S[at] = kInf;
      best = kInf;
      at = kNone;
      for (uint32_t i = lane; i < cnt; i += kWave) {
        const uint64_t v = S[i];
        if (v < best) {
          best = v;
          at = i;
        }
      }
    }
  }
  if ((uint32_t)lane < k) {
    out_ids[lane] = mine == kInf ? kNone : key_id(mine);
    out_d[lane] = mine == kInf ? __uint_as_float(0x7F800000u) : key_dist(mine);
  }
}

// Partial selection sort in global memory: C[0..kk) become the kk smallest
// of C[0..n), ascending.  For re-ranks too large for LDS (rare: an
// expansion count far above L); one wave, with a device fence per round so
// every lane sees lane 0's swap.
__device__ void global_select(uint64_t* C, uint32_t n, uint32_t kk, int lane) {
  for (uint32_t r = 0; r < kk && r < n; ++r) {
    uint64_t best = kInf;
    uint32_t at = kNone;
    for (uint32_t i = r + lane; i < n; i += kWave) {
      const uint64_t v = C[i];
      if (v < best) {
        best = v;
        at = i;
      }
    }
    const uint64_t m = wave_min64(best);
    const uint64_t who = __ballot(best == m && at != kNone);
    const uint32_t src = first_of(at, who);
    if (lane == 0 && src != kNone && src != r) {
      const uint64_t t = C[r];
      C[r] = m;
      C[src] = t;
    }
    __threadfence();
    __syncthreads();
  }
}

// The kq-th smallest of the distinct keys S[i], i < cnt (kq <= cnt), by kq
// rounds of a wave minimum over per-lane minima (best/at as in
// select_and_emit); the keys taken are overwritten with kInf.
__device__ uint64_t kth_key(uint64_t* S, uint32_t cnt, uint32_t kq,
                            uint64_t best, uint32_t at, int lane) {
  uint64_t m = kInf;
  for (uint32_t r = 0; r < kq; ++r) {
    m = wave_min64(best);
    if (m == kInf) break;
    if (best == m) {
      S[at] = kInf;
      best = kInf;
      at = kNone;
      for (uint32_t i = lane; i < cnt; i += kWave) {
        const uint64_t v = S[i];
        if (v < best) {
          best = v;
          at = i;
        }
      }
    }
  }
  return m;
}

// Squared distance between a bfloat16 row and the FP32 query, summed in
// FP32 over the coordinates in order (no FMA), the row read in one round
// trip.
template <int D>
__device__ __forceinline__ float bf16_dist(const uint16_t* __restrict__ row,
                                           const float* __restrict__ q) {
  static_assert(D % 8 == 0, "bfloat16 rows are read 16 bytes at a time");
  const uint4* x = reinterpret_cast<const uint4*>(row);
  uint4 v[D / 8];
#pragma unroll
  for (int c = 0; c < D / 8; ++c) v[c] = x[c];
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < D / 8; ++c) {
    const uint32_t w[4] = {v[c].x, v[c].y, v[c].z, v[c].w};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const uint32_t h = (w[t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
      const float xb = __uint_as_float(h << 16);
      const float diff = xb - q[8 * c + t];
      const float sq = diff * diff;
      acc = acc + sq;
    }
  }
  return acc;
}

// The re-rank of float data from bfloat16 rows with an FP32 recheck (the
// precision form's re-rank; the paper's is FP32, section "Re-ranking").
// For each candidate, D~ = bf16_dist and B = its row's sum of squares give
// the band E = 2^-6 sqrt(B D~) + 2^-15 B + 2^-12 D~, which bounds the gap
// between D~ and the candidate's canonical FP32 distance (the rounding of
// the row to bfloat16 moves the exact distance by at most
// 2v sqrt(B D~) + v^2 B, v = 2^-8 / (1 - 2^-8), by Cauchy-Schwarz, and the
// FP32 sums of d <= 1024 squares are within 6.2e-5 relative; every term of
// E is twice that).  tau = the kq-th smallest upper bound D~ + E; only the
// candidates whose lower bound D~ - E is <= tau can be among the kq nearest,
// and those get their FP32 distance; the kq nearest of them by (distance,
// id) are the FP32 re-rank's answer.  S holds the nc candidates' keys (id
// in the low bits); it and the two arrays behind it (2 * pow2ceil(nc) keys
// in all) are LDS.  Returns the number recomputed in FP32.  Out of line:
// its registers stay out of the search loop's allocation.
template <int D>
__device__ __attribute__((noinline)) uint32_t rerank_bf16(
    const float* __restrict__ base, const uint16_t* __restrict__ base16,
    const float* __restrict__ norm16, uint64_t* S, uint32_t nc, uint32_t kq,
    const float* q, uint32_t* oid, float* od, int lane) {
  const uint32_t P = pow2ceil_dev(nc);
  uint32_t* Id = reinterpret_cast<uint32_t*>(S + P);
  float* Lo = reinterpret_cast<float*>(Id + P);
  uint64_t best = kInf;
  uint32_t at = kNone;
#pragma unroll 1
  for (uint32_t i = lane; i < nc; i += kWave) {
    const uint32_t id = key_id(S[i]);
    const float dt = bf16_dist<D>(base16 + (size_t)id * D, q);
    const float nb = norm16[id];
    const float e1 = __builtin_sqrtf(nb * dt) * 0.015625f;   // 2^-6
    const float e2 = nb * 3.0517578125e-05f;                 // 2^-15
    const float e3 = dt * 2.44140625e-04f;                   // 2^-12
    const float E = (e1 + e2) + e3;
    const float lo = dt - E;
    const uint64_t key = make_key(dt + E, id);
    Id[i] = id;
    Lo[i] = lo > 0.0f ? lo : 0.0f;
    S[i] = key;
    if (key < best) {
      best = key;
      at = i;
    }
  }
  __syncthreads();
  float tau = __uint_as_float(0x7F800000u);
  if (nc > kq) {
    uint64_t tk;
    if (kq <= kWave) {
      tk = kth_key(S, nc, kq, best, at, lane);
    } else {
      for (uint32_t i = nc + lane; i < P; i += kWave) S[i] = kInf;
      __syncthreads();
      lds_sort(S, P, lane);
      tk = S[kq - 1];
    }
    tau = key_dist(tk);
  }
  __syncthreads();
  best = kInf;
  at = kNone;
  uint32_t cnt = 0;
#pragma unroll 1
  for (uint32_t i = lane; i < nc; i += kWave) {
    uint64_t key = kInf;
    if (Lo[i] <= tau) {
      const uint32_t id = Id[i];
      key = make_key(exact_dist<kF32, D, true>(base, id,
                                                reinterpret_cast<const
                                                unsigned char*>(q), 0),
                     id);
      ++cnt;
    }
    S[i] = key;
    if (key < best) {
      best = key;
      at = i;
    }
  }
  __syncthreads();
  if (kq <= kWave)
    select_and_emit(S, nc, kq, best, at, oid, od, lane);
  else
    sort_and_emit(S, nc, kq, oid, od, lane);
  // the count, summed over the wave
  uint32_t tot = cnt;
  tot += dpp<0x111>(0u, tot);
  tot += dpp<0x112>(0u, tot);
  tot += dpp<0x114>(0u, tot);
  tot += dpp<0x118>(0u, tot);
  tot += dpp<0x142, 0xA>(0u, tot);
  tot += dpp<0x143, 0xC>(0u, tot);
  return __builtin_amdgcn_readlane(tot, kWave - 1);
}

}  // namespace

// Arguments of one search launch (the same struct in every translation
// unit that includes this header).
struct SearchArgs {
  const void* base;
  const unsigned char* rows;  // packed rows: ids, then the neighbours' codes
  const uint8_t* codes;
  const float* cb;
  const uint32_t* hadj;  // host-resident adjacency [n][R], or null
  const unsigned char* queries;
  uint64_t nq;
  uint32_t n, R, medoid;
  uint32_t row_stride, row_ids;  // bytes per row; bytes of the id part
  uint32_t k, Lcap, c_max, iter_cap;
  uint32_t lblock;   // worklist entries per lane in a super-row, <= kPer
  uint32_t lrow;     // worklist buffer entries: Lcap rounded up to 64*lblock
  uint32_t region0;  // bytes of the table region (re-rank keys reuse it
                     // together with the worklist buffer)
  uint32_t s_cap;    // keys that fit there: (region0 + 8 * lrow) / 8, or
                     // 0 to make the re-rank select in global memory
  uint32_t* out_ids;   // [nq][k]: k is the row stride
  float* out_dists;
  // optional per-query worklist size and k (mixed batches): L_q in [1,
  // Lcap] and k_q in [1, min(k, L_q)] (clamped into range); the iteration
  // cap and c_max then follow L_q as their defaults do
  const uint32_t* qL;
  const uint32_t* qk;
  uint32_t* out_cand;
  uint32_t cand_stride;
  uint32_t* out_counters;
  uint64_t* out_times;
  uint32_t* out_phases;  // [nq][kPhases] (the timed variant only)
  uint64_t* cscratch;
  uint32_t* qcounter;
  uint32_t* bloom;        // null, or [grid][kBloomZ] filter entries
  uint32_t* bloom_epoch;  // [grid]
  // null, or a stop request in host memory (coherent, mapped): polled at
  // every query's start and every kAbortPoll expansions; abort_fired is
  // set when a query is cut short or skipped because of it
  const uint32_t* abort_flag;
  uint32_t* abort_fired;
  // float data only: base rows in bfloat16 and their sums of squares, for
  // the re-rank with an FP32 recheck (null: the exact FP32 re-rank)
  const uint16_t* base16;
  const float* norm16;
  // exact seen-set (the seen-bitmap variant only): per resident wave one
  // bit per node, seen_words words, all zero between queries; and a log of
  // the ids whose bits the current query set, kSeenLog entries per wave
  uint32_t* seen;
  uint32_t* seen_log;
  uint32_t seen_words;
  uint32_t seen_cap;  // ids a query may log, <= kSeenLog
  // null, or [nq][m][256] FP32 tables built beforehand (e.g. by BF16 MFMA):
  // each query's table is taken from here instead of being built
  const float* tables;
  // null, or [nq]: the order in which the waves take the queries (query
  // order[t] is the t-th taken); results stay in each query's own row
  const uint32_t* order;
  // exact distances with the set union: a direct-mapped cache of seen ids
  // in LDS at byte cache_off, cache_slots entries (a power of two, 0 =
  // none), slot of id x = (x * kCacheMul) >> cache_shift
  uint32_t cache_off, cache_slots, cache_shift;
};

namespace {

// The worklist is handled in super-rows of 64*B entries, B = ceil(L/64)
// capped at kPer; inside one, lane l owns the B entries
// [base + B*l, base + B*l + B).  L <= 256 is a single super-row.
constexpr int kPer = 4;

// Expansions between two readings of the stop request: a reading crosses
// the host link, so it is rare and issued well before it is needed.
constexpr uint32_t kAbortPoll = 64;

// The host's stop request, read past every cache; the same word on every
// lane, returned wave-uniform.
__device__ __forceinline__ uint32_t abort_requested(const uint32_t* flag) {
  const uint32_t v =
      __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  return __builtin_amdgcn_readfirstlane(v);
}

// Records on the host that a query stopped because of the request.
__device__ __forceinline__ void abort_record(uint32_t* fired, int lane) {
  if (lane == 0)
    __hip_atomic_store(fired, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Adjacency row of node u and, in the same row, the codes of its
// neighbours: one coalesced load per lane, no dependent gather.  With a
// host-resident adjacency only the ids are requested here (4R bytes across
// the host link); gather_codes fetches the codes once they have arrived.
// CODES = false (exact distances) requests the ids alone.  Every lane
// loads (lanes past R repeat slot R-1), so no lane-dependent branch joins
// the two forms; the caller applies row_mask once the row is in.
template <int M, bool CODES, bool HOST>
__device__ __forceinline__ void load_row(const SearchArgs& a, uint32_t u,
                                         int lane, uint32_t& nb,
                                         uint4 (&code)[M / 16]) {
  const uint32_t l = min((uint32_t)lane, a.R - 1);
  if constexpr (HOST) {
    nb = a.hadj[(size_t)u * a.R + l];
    return;
  }
  const unsigned char* row = a.rows + (size_t)u * a.row_stride;
  nb = reinterpret_cast<const uint32_t*>(row)[l];
  if (!CODES) return;
  const uint4* c = reinterpret_cast<const uint4*>(row + a.row_ids + l * M);
#pragma unroll
  for (int i = 0; i < M / 16; ++i) code[i] = c[i];
}

// kPer consecutive worklist keys from p (LDS, 8-byte aligned) in one batch
// of reads, with no branch between them.
__device__ __forceinline__ void load_block(const uint64_t* p,
                                           uint64_t (&x)[kPer]) {
#pragma unroll
  for (int t = 0; t < kPer; ++t) x[t] = p[t];
}

// Merge of the live new keys into the worklist (section "Parallel Merge":
// position = own index + rank in the other list), in place.  Lc: the
// worklist (Llen entries in super-rows of sup = 64*B, lane l owning B
// consecutive entries of each); keep / kk / r: this lane's live key and
// its worklist rank; idx: its index among the nv live keys (u* is
// already marked visited in the list).  A new key's position is r + (live
// keys below it); worklist entry j moves right by the live keys whose
// rank is <= j, a prefix of the byte histogram H of live ranks over
// super-rows s0 .. nsup-1 (NS = 1 when the worklist is a single
// super-row).  Every LDS read goes out before the first write, so entries
// move in place; a write with nothing to store goes to the lane's own
// slot of Nb, whose live keys are no longer needed, instead of behind a
// branch.  Slots of a block past the list are moved too: every live rank
// is below them, so they land at or past the new end (and before Lq),
// where nothing reads them.
template <int NS>
__device__ __forceinline__ void merge_live(
    uint64_t* Lc, uint64_t* Nb, uint32_t* Hw, int lane, uint32_t B,
    uint32_t sup, uint32_t Lq, uint32_t nsup, uint32_t s0, bool keep,
    uint64_t kk, uint32_t idx, uint32_t r, uint32_t nv) {
  uint64_t v[NS][kPer];
  uint32_t o[NS];  // this lane's first position per super-row (also its
                   // byte in H)
#pragma unroll
  for (int sr = 0; sr < NS; ++sr) {
    // super-rows past the list read super-row 0 again (unused); only the
    // super-rows that move (s0 .. nsup-1) are read
    o[sr] = (NS == 1 || (uint32_t)sr < nsup ? sr * sup : 0u) + B * lane;
    if (NS == 1 || ((uint32_t)sr >= s0 && (uint32_t)sr < nsup))
      load_block(Lc + o[sr], v[sr]);
  }
  if (keep) {
    Nb[idx] = kk;  // the live keys, compacted
    atomicAdd(&Hw[r >> 2], 1u << (8 * (r & 3)));
  }
  if (lane < 4) Nb[nv + lane] = kInf;  // pad to a multiple of 4
  __syncthreads();
  // this lane's B histogram bytes per super-row, from the two words
  // holding them (bytes past Llen count keys appended after every entry
  // or are zero; they move no entry)
  uint32_t w0[NS], w1[NS];
#pragma unroll
  for (int sr = 0; sr < NS; ++sr) {
    w0[sr] = Hw[o[sr] >> 2];
    w1[sr] = Hw[(o[sr] >> 2) + 1];
  }
  // rank among the live keys (their count below mine)
  uint32_t rn = 0;
  for (uint32_t j = 0; j < nv; j += 4) {
    const uint64_t x0 = Nb[j], x1 = Nb[j + 1], x2 = Nb[j + 2], x3 = Nb[j + 3];
    rn += (x0 < kk) + (x1 < kk) + (x2 < kk) + (x3 < kk);
  }
  const uint32_t bmask = B < 4 ? (1u << (8 * B)) - 1u : ~0u;
  // this lane's live-key count per super-row, one byte each: a count, and
  // any sum of them over lanes, is at most nv <= 64, so one scan of the
  // packed word scans every super-row at once with no carry between bytes
  static_assert(NS <= 4, "one byte per super-row");
  uint32_t hb[NS];
  uint32_t tot = 0;
#pragma unroll
  for (int sr = 0; sr < NS; ++sr) {
    const bool act = (uint32_t)sr < nsup && (uint32_t)sr >= s0;
    hb[sr] = act ? __builtin_amdgcn_alignbyte(w1[sr], w0[sr], o[sr] & 3u) &
                       bmask
                 : 0u;
    tot |= __builtin_amdgcn_udot4(hb[sr], 0x01010101u, 0u, false) << (8 * sr);
  }
  const uint32_t excl = wave_exclusive_scan(tot);
  // byte sr of carry: the live keys of the super-rows before sr
  const uint32_t carry =
      __builtin_amdgcn_readlane(excl + tot, kWave - 1) * 0x01010100u;
  uint32_t shift0[NS];
#pragma unroll
  for (int sr = 0; sr < NS; ++sr)
    shift0[sr] = __builtin_amdgcn_ubfe(carry, 8 * sr, 8) +
                 __builtin_amdgcn_ubfe(excl, 8 * sr, 8);
#pragma unroll
  for (int sr = 0; sr < NS; ++sr) {
    if ((uint32_t)sr >= nsup || (uint32_t)sr < s0) continue;
    const uint32_t j0 = sr * sup + B * lane;
    uint32_t p = j0 + shift0[sr];
    // with several super-rows B = kPer; a super-row whose entries all stay
    // below Lq after moving right by at most nv needs no test per entry
    if (NS > 1 && (sr + 1) * sup + nv <= Lq) {
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        p += __builtin_amdgcn_ubfe(hb[sr], 8 * t, 8);
        Lc[p] = v[sr][t];
        ++p;
      }
      continue;
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      p += __builtin_amdgcn_ubfe(hb[sr], 8 * t, 8);
      const bool ok = (NS > 1 || (uint32_t)t < B) && p < Lq;
      uint64_t* dst = ok ? Lc + p : Nb + lane;
      *dst = v[sr][t];
      ++p;
    }
  }
  if (keep && r + rn < Lq) Lc[r + rn] = kk;
}

// The merge of a single live key x of worklist rank r (wave-uniform; the
// usual merge): entries r .. Lq-2 move right by one, the entry at Lq-1 of
// a full list drops out, and x takes position r.  No histogram and no
// ranking among live keys; the same in-place order of reads before writes
// as merge_live, and the same spare slot of Nb for a lane with nothing to
// store.
template <int NS>
__device__ __forceinline__ void merge_one(uint64_t* Lc, uint64_t* Nb,
                                          int lane, uint32_t B, uint32_t sup,
                                          uint32_t Lq, uint32_t nsup,
                                          uint32_t s0, uint32_t r,
                                          uint64_t x) {
  uint64_t v[NS][kPer];
#pragma unroll
  for (int sr = 0; sr < NS; ++sr) {
    const uint32_t o = (NS == 1 || (uint32_t)sr < nsup ? sr * sup : 0u) +
                       B * lane;
    if (NS == 1 || ((uint32_t)sr >= s0 && (uint32_t)sr < nsup))
      load_block(Lc + o, v[sr]);
  }
#pragma unroll
  for (int sr = 0; sr < NS; ++sr) {
    if ((uint32_t)sr >= nsup || (uint32_t)sr < s0) continue;
    const uint32_t j0 = sr * sup + B * lane;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const uint32_t j = j0 + t;
      const bool ok = (NS > 1 || (uint32_t)t < B) && j >= r && j + 1 < Lq;
      uint64_t* dst = ok ? Lc + j + 1 : Nb + lane;
      *dst = v[sr][t];
    }
  }
  if (lane == 0) Lc[r] = x;
}

// Lanes past R hold no neighbour.
__device__ __forceinline__ uint32_t row_mask(const SearchArgs& a, int lane,
                                             uint32_t nb) {
  return (uint32_t)lane < a.R ? nb : kNone;
}

// The paper's visited filter ("Parallel Filtering of Visited Neighbours";
// z and the two FNV-1a hashes in "Algorithm Parameters").  FNV-1a-32: per
// byte, xor it into the state, then multiply by the FNV prime; the two
// hashes run over the id's four little-endian bytes from offset bases
// kFnvBasis and kFnvBasis ^ kBloomSalt and are taken mod z.
//
// Each entry holds a 32-bit tag instead of a bool: epoch field (bits 31-20,
// kBloomEpochs - query epoch, so the filters of earlier queries read as
// larger), expansion (bits 19-6; 0 for the medoid) and lane (bits 5-0).
// An entry counts as set for lane j of expansion e iff it holds a tag below
// j's own: set by an earlier expansion of this query, or by an earlier lane
// of this row.  Every lane takes atomicMin with its tag on both entries and
// gets the previous value back; the earlier lane whose update lands after a
// later lane's sees that lane's tag, and passes the fact on (below).
constexpr uint32_t kBloomZ = 399887u;
constexpr uint32_t kFnvBasis = 0x811C9DC5u;
constexpr uint32_t kFnvPrime = 0x01000193u;
constexpr uint32_t kBloomSalt = 0xA5A5A5A5u;
constexpr uint32_t kBloomEpochs = 4095u;  // queries per filter clear

__device__ __forceinline__ void bloom_slots(uint32_t x, uint32_t& h1,
                                            uint32_t& h2) {
  uint32_t a = kFnvBasis, b = kFnvBasis ^ kBloomSalt;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t c = (x >> (8 * i)) & 0xFFu;
    a = (a ^ c) * kFnvPrime;
    b = (b ^ c) * kFnvPrime;
  }
  h1 = a % kBloomZ;
  h2 = b % kBloomZ;
}

// Touches node u's packed row, one word per lane spread over the part that
// load_row reads: the row comes into the caches while the current
// neighbours are scored, so that load_row, if u is chosen, finds it there.
// With a host-resident adjacency u's codes in device memory are touched
// instead (no host-link traffic; the load only keeps the loads outstanding
// the same on every path).  `touched` receives the word; the caller
// consumes the previous one (keep_alive) once it is long complete, which
// keeps each load from being dropped.
// Algorithm 2's test-then-set for this lane's neighbour nb, issued as one
// atomicMin per entry (the previous values come back in o1, o2).
__device__ __forceinline__ void bloom_update(uint32_t* bf, uint32_t btop,
                                             uint32_t iters, int lane,
                                             uint32_t nb, uint32_t& h1,
                                             uint32_t& h2, uint32_t& tag,
                                             uint32_t& o1, uint32_t& o2) {
  if (!bf) return;
  bloom_slots(nb, h1, h2);
  tag = btop | (iters << 6) | (uint32_t)lane;
  if (nb != kNone) {
    o1 = atomicMin(bf + h1, tag);
    o2 = atomicMin(bf + h2, tag);
  }
}

// Exact seen-set (Algorithm 2's visited filter without false positives):
// one bit per node in the wave's bitmap.  Each neighbour of an expanded row
// takes one atomicOr with its bit, which sets it and returns the word as it
// was: a clear bit means the neighbour is new to the query.  While the log
// has room for a whole row the bit is set and new ids are logged; after
// that the word is only read (atomicOr with 0), so a new neighbour counts
// as unseen again later, which the set union in the worklist resolves.  A
// set bit is therefore always a node seen before, and dropping it changes
// nothing: it is in the worklist already, or its key lies past the last
// entry, which never grows once the worklist is full.  At the query's end
// the logged words are stored as zero, which leaves the bitmap clear.
constexpr uint32_t kSeenLog = 8192u;  // logged ids per wave

// Multiplier of the seen-id cache's slot hash (exact distances): the top
// bits of id * 2654435761 (Knuth's multiplicative hashing, 2^32 over the
// golden ratio).
constexpr uint32_t kCacheMul = 2654435761u;

enum Filter : int { kFiltUnion = 0, kFiltBloom = 1, kFiltSeen = 2 };

__device__ __forceinline__ uint32_t seen_update(uint32_t* sb, uint32_t nb,
                                                bool set) {
  if (nb == kNone) return ~0u;  // an empty slot reads as seen
  return atomicOr(sb + (nb >> 5), set ? 1u << (nb & 31u) : 0u);
}

template <int M, bool CODES, bool HOST>
__device__ __forceinline__ void touch_row(const SearchArgs& a, uint32_t u,
                                          int lane, uint32_t& touched) {
  const uint32_t bytes = a.row_ids + (CODES ? a.R * M : 0u);
  const uint32_t step = (bytes / kWave) & ~3u;
  const unsigned char* p =
      HOST ? a.codes + (size_t)u * M
           : a.rows + (size_t)u * a.row_stride + lane * step;
  touched = *reinterpret_cast<const uint32_t*>(p);
}

// An empty statement that uses v: the compiler must have v (a load's
// result) at this point.
__device__ __forceinline__ void keep_alive(uint32_t v) {
  asm volatile("" ::"v"(v));
}

// Waves per SIMD that the table alone still lets share a CU's 160 KB of
// LDS: the register allocator may spend up to that share, so it keeps more
// LDS reads in flight where few waves are resident anyway.
constexpr int max_waves_per_simd(int table_bytes) {
  const int per_cu = (160 * 1024) / (table_bytes + 1280);
  const int w = (per_cu + 3) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// Codes of neighbour nb from the [n][m] code array in device memory (host-
// resident adjacency only; the packed rows carry them otherwise).
template <int M, bool HOST>
__device__ __forceinline__ void gather_codes(const SearchArgs& a, uint32_t nb,
                                             uint4 (&code)[M / 16]) {
  if (HOST && nb != kNone) {
    const uint4* c = reinterpret_cast<const uint4*>(a.codes + (size_t)nb * M);
#pragma unroll
    for (int i = 0; i < M / 16; ++i) code[i] = c[i];
  }
}

// Phases of a query that the timed variant reports (out_phases), in
// shader-clock cycles (s_memtime): the table and the worklist's start, then
// summed over the expansions: waiting for the row, scoring the neighbours,
// ranking them in the worklist (with the visited test), choosing the next
// node and requesting its row, merging; then the re-rank.
constexpr int kPhases = 7;

__device__ __forceinline__ uint64_t phase_clock() {
  return __builtin_amdgcn_s_memtime();
}

// HOST: adjacency rows in pinned host memory (a.hadj), the codes gathered
// from device memory.  FILT: the visited test besides the set union in the
// worklist: none, the paper's Bloom filter (a.bloom), or the exact seen
// bitmap (a.seen), which skips the worklist rank of a row whose neighbours
// were all seen.  Each is its own instantiation, so that no form's extra
// loads and atomics change where the others wait for memory.  PHASES: the
// timed variant, which adds up shader-clock cycles per phase of each query
// (out_phases) and is otherwise the same search.
template <int DT, int M, int DS, int TT, bool HOST, int FILT, bool PHASES>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(
    TT == kTabExact ? 4 : 1, max_waves_per_simd(table_bytes<TT>(M)))))
void search_kernel(SearchArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool BLOOM = FILT == kFiltBloom;
  constexpr bool SEEN = FILT == kFiltSeen;
  constexpr int D = M * DS;
  constexpr int kTableBytes = table_bytes<TT>(M);
  constexpr bool kExact = TT == kTabExact;
  // exact distances with the set union: the seen-id cache in LDS
  constexpr bool kCache = kExact && FILT == kFiltUnion;
  const int lane = threadIdx.x;
  void* T = smem;
  float* lo = reinterpret_cast<float*>(smem + kTableBytes);  // U8 offsets
  uint64_t* S = reinterpret_cast<uint64_t*>(smem);  // re-rank keys
  const uint32_t B = a.lblock;
  const uint32_t sup = kWave * B;  // super-row size
  // the worklist (merged in place), the live new keys, and a histogram of
  // the live keys' worklist ranks: one byte per position (a count is at
  // most 64), added to as 32-bit words
  uint64_t* Lc = reinterpret_cast<uint64_t*>(smem + a.region0);  // lrow
  uint64_t* Nb = Lc + a.lrow;                                     // kWave + 4
  uint8_t* H = reinterpret_cast<uint8_t*>(Nb + kWave + 4);        // lrow + 4
  uint32_t* Hw = reinterpret_cast<uint32_t*>(H);
  uint32_t* const Sc = reinterpret_cast<uint32_t*>(smem + a.cache_off);
  uint64_t* C = a.cscratch + (size_t)blockIdx.x * a.iter_cap;
  for (uint32_t t = lane; t < (a.lrow + 4) / 4; t += kWave) Hw[t] = 0u;

  for (;;) {
    uint32_t qi = 0;
    if (lane == 0) qi = atomicAdd(a.qcounter, 1u);
    qi = __builtin_amdgcn_readfirstlane(qi);
    if (qi >= a.nq) {
      // the last workgroup out returns both counters to zero for the next
      // launch (no reset kernel or memset on the stream)
      if (lane == 0) {
        __threadfence();
        if (atomicAdd(a.qcounter + 1, 1u) == gridDim.x - 1) {
          atomicExch(a.qcounter, 0u);
          atomicExch(a.qcounter + 1, 0u);
        }
      }
      break;
    }
    // the queries are taken in a.order when it is given (an entry past the
    // batch takes the last query, searched twice with the same result)
    if (a.order)
      qi = min(__builtin_amdgcn_readfirstlane(a.order[qi]),
               (uint32_t)(a.nq - 1));
    const uint64_t t_begin = a.out_times ? wall_clock64() : 0;
    if (a.abort_flag && abort_requested(a.abort_flag)) {
      // stopped: this query is not searched; its row is padding, status 2
      uint32_t* oid = a.out_ids + (size_t)qi * a.k;
      float* od = a.out_dists + (size_t)qi * a.k;
      for (uint32_t i = lane; i < a.k; i += kWave) {
        oid[i] = kNone;
        od[i] = __uint_as_float(0x7F800000u);
      }
      if (a.out_counters && lane < 4)
        a.out_counters[qi * 4 + lane] = lane == 1 ? 2u : 0u;
      if (a.out_cand)
        for (uint32_t i = lane; i < a.cand_stride; i += kWave)
          a.out_cand[(size_t)qi * a.cand_stride + i] = kNone;
      if (a.out_times && lane == 0) {
        a.out_times[qi * 2] = t_begin;
        a.out_times[qi * 2 + 1] = wall_clock64();
      }
      abort_record(a.abort_fired, lane);
      continue;
    }
    const unsigned char* q = a.queries + (size_t)qi * D * Elem<DT>::size;
    uint64_t ph[kPhases] = {0, 0, 0, 0, 0, 0, 0};
    uint64_t tp = PHASES ? phase_clock() : 0, t4 = 0;
    // this query's worklist size, result count, iteration cap and c_max
    uint32_t Lq = a.Lcap, kq = a.k, capq = a.iter_cap, cmq = a.c_max;
    if (a.qL) {
      Lq = min(max(a.qL[qi], 1u), a.Lcap);
      capq = min(max(4u * Lq, Lq + 64u), a.iter_cap);
      cmq = 4u * Lq;
    }
    if (a.qk) kq = min(max(a.qk[qi], 1u), min(a.k, Lq));

    // stage 1: the table (the previous query's re-rank is done with S)
    __syncthreads();
    const uint32_t s = a.medoid;
    // Bloom filter: this query's epoch (the wave's entries are cleared when
    // the epochs run out), and the medoid set first, as expansion 0
    uint32_t* const bf =
        BLOOM ? a.bloom + (size_t)blockIdx.x * kBloomZ : nullptr;
    uint32_t btop = 0;
    if constexpr (BLOOM) {
      uint32_t ep = 0;
      if (lane == 0) ep = atomicAdd(a.bloom_epoch + blockIdx.x, 1u) + 1u;
      ep = __builtin_amdgcn_readfirstlane(ep);
      if (ep > kBloomEpochs) {
        for (uint32_t i = lane; i < kBloomZ; i += kWave) bf[i] = 0xFFFFFFFFu;
        if (lane == 0) atomicExch(a.bloom_epoch + blockIdx.x, 1u);
        ep = 1u;
      }
      btop = (kBloomEpochs - ep) << 20;
      if (lane == 0) {
        uint32_t h1, h2;
        bloom_slots(s, h1, h2);
        atomicMin(bf + h1, btop);
        atomicMin(bf + h2, btop);
      }
      // clears and the medoid's tags are in place before any row's update
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      __threadfence_block();
    }
    // seen bitmap: the previous query's clearing stores are complete, then
    // the medoid is the first id seen and logged
    uint32_t* const sb =
        SEEN ? a.seen + (size_t)blockIdx.x * a.seen_words : nullptr;
    uint32_t* const slog =
        SEEN ? a.seen_log + (size_t)blockIdx.x * kSeenLog : nullptr;
    uint32_t nlog = 0;
    if constexpr (SEEN) {
      __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      if (lane == 0) {
        atomicOr(sb + (s >> 5), 1u << (s & 31u));
        slog[0] = s;
      }
      nlog = 1;
    }
    // seen-id cache: cleared, then the medoid is the first id in it
    if constexpr (kCache) {
      if (a.cache_slots) {
        for (uint32_t i = 4u * lane; i < a.cache_slots; i += 4u * kWave)
          *reinterpret_cast<uint4*>(Sc + i) =
              make_uint4(kNone, kNone, kNone, kNone);
        if (lane == 0) Sc[(s * kCacheMul) >> a.cache_shift] = s;
      }
    }
    // constant term of integer exact distances (the PQ forms compute it
    // after the search, so the query is not held through the loop)
    int32_t qq = 0;
    uint4 qc = make_uint4(0u, 0u, 0u, 0u);  // this lane's query chunk
    if constexpr (kExact) {
      qq = query_sq<DT, D>(q);
      if constexpr (DT != kF32) {
        constexpr int CH = D / 16;
        constexpr int G = CH <= 2 ? 2 : (CH <= 4 ? 4 : 8);
        const int c = lane % G;
        if (c < CH) qc = reinterpret_cast<const uint4*>(q)[c];
      }
    }
    uint32_t nb;
    uint4 code[M / 16];
    uint4 scode[M / 16];  // the medoid's own code (PQ forms)
    if constexpr (!kExact) {
      QueryLanes<DT, D> Q;
      Q.load(q, lane);
#pragma unroll
      for (int i = 0; i < M / 16; ++i)
        scode[i] = reinterpret_cast<const uint4*>(a.codes + (size_t)s * M)[i];
      load_row<M, true, HOST>(a, s, lane, nb, code);  // in flight meanwhile
      build_table_q<DT, M, DS, TT>(
          Q, a.cb, a.tables ? a.tables + (size_t)qi * M * 256 : nullptr, T,
          lo, lane);
    } else {
      load_row<M, false, HOST>(a, s, lane, nb, code);
    }
    __syncthreads();

    // stage 2: L = [(dist(s), s)]
    float d0;
    if constexpr (kExact) {
      d0 = exact_dist<DT, D>(a.base, s, q, qq);
    } else {
      d0 = adc_codes<M, TT>(scode);
    }
    uint64_t curkey = make_key(d0, s);
    if (lane == 0) Lc[0] = curkey;
    uint32_t Llen = 1, cur = 0, iters = 0, status = 0;
    // the rank's first-level entries (255, 511, 767, clamped to the last
    // one), the same for every key until the list changes: read after each
    // merge, off the rank's path, and only once the list passes 256
    // entries (the rank skips the level below that)
    uint64_t top[3] = {curkey, curkey, curkey};
    uint32_t touched = 0;  // result of the last touch_row (never read)
    // the expanded keys, written to C 64 at a time: lane e holds that of
    // expansion e mod 64 until its group of 64 is stored
    uint64_t ckey = 0;
    // the last reading of the stop request (taken every kAbortPoll
    // expansions, used one expansion later)
    uint32_t abw = 0;
    __syncthreads();

    if constexpr (PHASES) {
      const uint64_t t = phase_clock();
      ph[0] = t - tp;
    }
    while (cur != kNone) {
      if (iters == capq) {
        status = 1;
        break;
      }
      if (abw) {
        status = 2;
        break;
      }
      if constexpr (PHASES) tp = phase_clock();
      // expand u* = Lc[cur]: mark visited, record it as a candidate
      if (lane == 0) Lc[cur] = curkey | 1ull;
      if ((uint32_t)lane == (iters & (kWave - 1))) ckey = curkey;
      if ((iters & (kWave - 1)) == kWave - 1) {
        C[iters - (kWave - 1) + lane] = ckey;
        // completed here: with a store outstanding among the row loads the
        // compiler can only wait for every access, the touch below included
        __builtin_amdgcn_s_waitcnt(kWaitVmem0);
      }
      ++iters;
      const uint32_t sbase = cur / sup * sup;
      const uint64_t last = Lc[Llen - 1];
      // the entry after u*: every entry before u* is visited, so when this
      // one is not, it is the first unvisited entry a (the usual case)
      const uint64_t nx = Lc[min(cur + 1, Llen - 1)];
      // it is usually the next node too: its row is touched below, after
      // this row's ids are in (when nx is visited or past the end the touch
      // is wasted, not wrong).  The previous touch was issued before this
      // row was requested, so it is complete.

      // distances of the neighbours (row of u*, loaded earlier)
      nb = row_mask(a, lane, nb);
      keep_alive(touched);
      // read the stop request now and then; the reading is complete by the
      // time the next row is, where the loop looks at it
      if (a.abort_flag && (iters & (kAbortPoll - 1)) == 1)
        abw = abort_requested(a.abort_flag);
      if constexpr (PHASES) {
        keep_alive(nb);
        const uint64_t t = phase_clock();
        ph[1] += t - tp;
        tp = t;
      }
      // exact distances: a neighbour whose id is in the seen-id cache was
      // seen before in this query, so the set union would drop it; its
      // base row is not read and it takes no part.  The others enter the
      // cache (replacing the id in their slot) and, for integer data, move
      // to the first lanes, so that loads of rows past them are not issued.
      uint64_t cmask = ~0ull;  // lanes with a neighbour to score
      uint32_t nlive = kWave;
      if constexpr (kCache) {
        if (a.cache_slots) {
          const uint32_t h = (nb * kCacheMul) >> a.cache_shift;
          const bool fresh = nb != kNone && Sc[h] != nb;
          if (fresh) Sc[h] = nb;
          cmask = __ballot(fresh);
          nlive = (uint32_t)__popcll(cmask);
          if constexpr (DT != kF32) {
            // fresh ids to lanes 0..nlive-1 in row order, the rest after
            // them (a permutation of the lanes)
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(cmask >> 32),
                __builtin_amdgcn_mbcnt_lo((uint32_t)cmask, 0u));
            const uint32_t dst =
                fresh ? below : nlive + ((uint32_t)lane - below);
            nb = (uint32_t)__builtin_amdgcn_ds_permute(
                (int)(dst * 4u), (int)(fresh ? nb : kNone));
            cmask = nlive == (uint32_t)kWave ? ~0ull : (1ull << nlive) - 1ull;
          } else if (!fresh) {
            nb = kNone;
          }
        }
      }
      // Bloom filter: both entries of each neighbour are updated with this
      // lane's tag below (after any code gather, so that the scoring waits
      // for neither); the previous values are used after the scoring
      uint32_t b1 = 0, b2 = 0, btag = 0, bo1 = ~0u, bo2 = ~0u;
      // seen bitmap: each neighbour's word as it was before this row set
      // its bit, back during the scoring (set only while the log has room)
      uint32_t sold = 0;
      const bool sset = nlog + kWave <= a.seen_cap;
      uint64_t key = kInf;
      if constexpr (kExact && DT != kF32) {
        bloom_update(bf, btop, iters, lane, nb, b1, b2, btag, bo1, bo2);
        if constexpr (SEEN) sold = seen_update(sb, nb, sset);
        touch_row<M, false, HOST>(a, key_id(nx), lane, touched);
        const float dq = coop_dist<DT, D>(a.base, nb, qc, qq, lane, nlive);
        key = nb != kNone ? make_key(dq, nb) : kInf;
      } else if constexpr (kExact) {
        bloom_update(bf, btop, iters, lane, nb, b1, b2, btag, bo1, bo2);
        if constexpr (SEEN) sold = seen_update(sb, nb, sset);
        touch_row<M, false, HOST>(a, key_id(nx), lane, touched);
        if (nb != kNone)
          key = make_key(exact_dist<DT, D, true>(a.base, nb, q, qq), nb);
      } else {
        gather_codes<M, HOST>(a, nb, code);
        // the codes are in before the filter's atomics go out: a wait for a
        // load with atomics outstanding waits for the atomics too
        if constexpr (BLOOM) {
#pragma unroll
          for (int i = 0; i < M / 16; ++i)
            keep_alive(code[i].x), keep_alive(code[i].y),
                keep_alive(code[i].z), keep_alive(code[i].w);
        }
        bloom_update(bf, btop, iters, lane, nb, b1, b2, btag, bo1, bo2);
        if constexpr (SEEN) sold = seen_update(sb, nb, sset);
        touch_row<M, true, HOST>(a, key_id(nx), lane, touched);
        // every lane sums (no branch): an empty slot has zero codes, a lane
        // past R reads table entries it then discards
        const uint64_t k2 = make_key(adc_codes<M, TT>(code), nb);
        key = nb != kNone ? k2 : kInf;
      }
      // a neighbour found in the seen-id cache, or whose seen bit was set,
      // is dropped before the worklist rank, which a row with no other
      // neighbour skips; new bits are logged (in row order) for the
      // clearing at the end
      uint64_t fresh_mask = cmask;
      if constexpr (SEEN) {
        const bool fresh = !((sold >> (nb & 31u)) & 1u);
        fresh_mask = __ballot(fresh);
        if (!fresh) key = kInf;
        if (sset) {
          const uint32_t at = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(fresh_mask >> 32),
              __builtin_amdgcn_mbcnt_lo((uint32_t)fresh_mask, 0u));
          if (fresh) slog[nlog + at] = nb;
          nlog += (uint32_t)__popcll(fresh_mask);
        }
      }

      if constexpr (PHASES) {
        keep_alive((uint32_t)key), keep_alive((uint32_t)(key >> 32));
        const uint64_t t = phase_clock();
        ph[2] += t - tp;
        tp = t;
      }
      // rank in the worklist; a node already in it is dropped (set union);
      // a key ranked past a full worklist is cut whatever the other new keys
      // are, so only the remaining ("live") keys take part in the merge.
      // No branch for empty slots: kInf ranks past the last entry, with no
      // entry equal to it, and is never kept.
      uint64_t ge = kInf;
      uint32_t r = Llen;
      if (fresh_mask) r = rank_in(a.region0, Llen, last, top, key, ge);
      bool keep = (ge >> 1) != (key >> 1) && r < Lq;
      if constexpr (BLOOM) {
        // an entry is set for this lane if it held a smaller tag: an
        // earlier expansion's or an earlier lane's that landed first
        bool c1 = bo1 < btag, c2 = bo2 < btag;
        // an earlier lane whose update landed after a later lane's got
        // that lane's tag back (same expansion, larger lane): the later
        // lane learns here that its entry was set before it
        const bool n1 = nb != kNone && (bo1 >> 6) == (btag >> 6) &&
                        (bo1 & 63u) > (uint32_t)lane;
        const bool n2 = nb != kNone && (bo2 >> 6) == (btag >> 6) &&
                        (bo2 & 63u) > (uint32_t)lane;
        uint64_t need = __ballot(n1 || n2);
        while (need) {
          const int i = __builtin_ctzll(need);
          need &= need - 1;
          const uint32_t f1 = __builtin_amdgcn_readlane((uint32_t)n1, i);
          const uint32_t f2 = __builtin_amdgcn_readlane((uint32_t)n2, i);
          const uint32_t t1 = __builtin_amdgcn_readlane(bo1, i);
          const uint32_t t2 = __builtin_amdgcn_readlane(bo2, i);
          const uint32_t p1 = __builtin_amdgcn_readlane(b1, i);
          const uint32_t p2 = __builtin_amdgcn_readlane(b2, i);
          if (f1 && (uint32_t)lane == (t1 & 63u)) {
            c1 = c1 || b1 == p1;
            c2 = c2 || b2 == p1;
          }
          if (f2 && (uint32_t)lane == (t2 & 63u)) {
            c1 = c1 || b1 == p2;
            c2 = c2 || b2 == p2;
          }
        }
        if (c1 && c2) keep = false;  // both entries set: counted as visited
      }
      const uint64_t kk = keep ? key : kInf;
      if constexpr (PHASES) {
        keep_alive((uint32_t)kk), keep_alive((uint32_t)(kk >> 32));
        const uint64_t t = phase_clock();
        ph[3] += t - tp;
        tp = t;
      }

      // next node, decided before the merge: the smaller of the first
      // unvisited worklist entry a and the best new key b.  a is never cut
      // when it is the smaller; b is cut when its worklist rank reaches L,
      // and then a is cut too.  Its merged position is a's index or b's rank.
      uint32_t apos = kNone;
      uint64_t akey = kInf;
      if (cur + 1 < Llen && !(nx & 1ull)) {
        apos = cur + 1;
        akey = nx;
      } else {
        // scan from the super-row holding u*.  Each lane reads kPer
        // entries at once whatever B is (no load waits behind a branch):
        // those past its B belong to the next lane or, for the last lane
        // of the last super-row, to the live-key buffer after the worklist,
        // so every read stays inside the LDS block; they are not used.
        uint32_t ja = kNone;
        uint64_t va = kInf;
        {
          uint64_t x[kPer];
          load_block(Lc + sbase + B * lane, x);
#pragma unroll
          for (int t = kPer - 1; t >= 0; --t) {
            const uint32_t j = sbase + B * lane + t;
            if ((uint32_t)t < B && j < Llen && j > cur && !(x[t] & 1ull)) {
              ja = j;
              va = x[t];
            }
          }
        }
        uint64_t am = __ballot(ja != kNone);
        for (uint32_t base = sbase + sup; !am && base < Llen; base += sup) {
          uint64_t x[kPer];
          load_block(Lc + base + B * lane, x);
#pragma unroll
          for (int t = kPer - 1; t >= 0; --t) {
            const uint32_t j = base + B * lane + t;
            if ((uint32_t)t < B && j < Llen && !(x[t] & 1ull)) {
              ja = j;
              va = x[t];
            }
          }
          am = __ballot(ja != kNone);
        }
        if (am) {
          apos = first_of(ja, am);
          akey = ((uint64_t)first_of((uint32_t)(va >> 32), am) << 32) |
                 first_of((uint32_t)va, am);
        }
      }
      // b, the best live key, has the smallest worklist rank rb of them
      // (ranks follow key order); live keys of equal rank fall between the
      // same two entries and are told apart by a wave minimum over those
      // lanes alone.  No live key (most expansions once the worklist is
      // full): b does not exist.
      const uint64_t km = __ballot(keep);
      uint64_t bkey = kInf;
      uint32_t rb = kNone;
      if (km) {
        rb = wave_min32(keep ? r : kNone);
        const uint64_t tie = __ballot(keep && r == rb);
        if ((tie & (tie - 1)) == 0) {
          const int l = __builtin_ctzll(tie);
          bkey = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(kk >> 32), l)
                  << 32) |
                 __builtin_amdgcn_readlane((uint32_t)kk, l);
        } else {
          bkey = wave_min64(keep && r == rb ? kk : kInf);
        }
      }
      uint32_t best = kNone;
      uint64_t bestkey = kInf;
      if (bkey < akey) {
        if (rb < Lq) {
          best = rb;
          bestkey = bkey;
        }
      } else if (akey != kInf) {
        best = apos;
        bestkey = akey;
      }
      // request the next row now; it arrives during the merge
      if (best != kNone)
        load_row<M, !kExact, HOST>(a, key_id(bestkey), lane, nb, code);
      else
        nb = kNone;
      if constexpr (PHASES) {
        t4 = phase_clock();
        ph[4] += t4 - tp;
      }

      const uint32_t nv = __popcll(km);
      if (nv == 0) {
        // nothing enters the worklist: it keeps its order, u* is already
        // marked, and the next node is the first unvisited entry
        cur = best;
        curkey = bestkey;
        __syncthreads();
        if constexpr (PHASES) ph[5] += phase_clock() - t4;
        continue;
      }
      // smallest worklist rank of a live key (b's): entries below it stay
      const uint32_t rmin = rb;
      const uint32_t idx = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
      // super-rows in use and the first one with a moving entry (Llen and
      // rmin are below 4 super-rows: B is capped so that L fits in kPer)
      const uint32_t nsup =
          1u + (Llen > sup) + (Llen > 2u * sup) + (Llen > 3u * sup);
      const uint32_t s0 = (rmin >= sup) + (rmin >= 2u * sup) +
                          (rmin >= 3u * sup);
      if (nv == 1) {
        // one live key: b, of rank rb (below Lq, as every live key's)
        if (nsup == 1)
          merge_one<1>(Lc, Nb, lane, B, sup, Lq, nsup, s0, rb, bkey);
        else
          merge_one<kPer>(Lc, Nb, lane, B, sup, Lq, nsup, s0, rb, bkey);
      } else {
        if (nsup == 1)
          merge_live<1>(Lc, Nb, Hw, lane, B, sup, Lq, nsup, s0, keep, kk,
                        idx, r, nv);
        else
          merge_live<kPer>(Lc, Nb, Hw, lane, B, sup, Lq, nsup, s0, keep, kk,
                           idx, r, nv);
        // clear the histogram bytes used (positions rmin .. Llen)
        for (uint32_t t = rmin / 4 + lane; t <= Llen / 4; t += kWave)
          Hw[t] = 0u;
      }
      Llen = min(Lq, Llen + nv);
      cur = best;
      curkey = bestkey;
      __syncthreads();
      if (Llen > 256) {
        top[0] = Lc[255];
        top[1] = Lc[min(511u, Llen - 1)];
        top[2] = Lc[min(767u, Llen - 1)];
      }
      if constexpr (PHASES) ph[5] += phase_clock() - t4;
    }
    if constexpr (PHASES) tp = phase_clock();

    // stage 3: re-rank the expanded nodes.  The last group of C is written
    // out; an agent-scope fence then also drops stale L1 lines.
    if ((iters & ~(kWave - 1u)) + lane < iters)
      C[(iters & ~(kWave - 1u)) + lane] = ckey;
    __threadfence();
    __syncthreads();
    if constexpr (SEEN) {
      // clear the words of every id this query set (the log is read after
      // the fence above); the stores complete before the next query's
      // first update
#pragma unroll 1
      for (uint32_t i0 = 0; i0 < nlog; i0 += 4 * kWave) {
        uint32_t id[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t i = i0 + u * kWave + lane;
          id[u] = i < nlog ? slog[i] : kNone;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (id[u] != kNone) sb[id[u] >> 5] = 0u;
      }
    }
    if (a.out_counters && lane == 0) {
      a.out_counters[qi * 4 + 0] = iters;
      a.out_counters[qi * 4 + 1] = status;
      a.out_counters[qi * 4 + 2] = 0;
      a.out_counters[qi * 4 + 3] = 0;
    }
    if (a.out_cand)
      for (uint32_t i = lane; i < a.cand_stride; i += kWave)
        a.out_cand[(size_t)qi * a.cand_stride + i] =
            i < iters ? key_id(C[i]) : kNone;
    uint32_t nc = iters;
    uint32_t rechecked = 0;  // FP32 distances of the bfloat16 re-rank
    uint32_t* oid = a.out_ids + (size_t)qi * a.k;
    float* od = a.out_dists + (size_t)qi * a.k;
    if (status == 2) {
      // cut short by the stop request: no re-rank, the row is padding
      for (uint32_t i = lane; i < kq; i += kWave) {
        oid[i] = kNone;
        od[i] = __uint_as_float(0x7F800000u);
      }
      abort_record(a.abort_fired, lane);
    } else if constexpr (kExact) {
      // no re-rank: the worklist already ranks by exact distance
      for (uint32_t i = lane; i < kq; i += kWave) {
        const uint64_t key = i < Llen ? Lc[i] : kInf;
        oid[i] = key == kInf ? kNone : key_id(key);
        od[i] = key == kInf ? __uint_as_float(0x7F800000u) : key_dist(key);
      }
    } else if (qq = query_sq<DT, D>(q); pow2ceil_dev(nc) <= a.s_cap) {
      // sort in LDS (table region + worklist buffer, free now)
      if (nc > cmq) {
        // keep the c_max smallest (PQ distance, id)
        const uint32_t P = pow2ceil_dev(nc);
        for (uint32_t i = lane; i < P; i += kWave)
          S[i] = i < nc ? (C[i] & ~1ull) : kInf;
        __syncthreads();
        lds_sort(S, P, lane);
        nc = cmq;
      } else {
        for (uint32_t i = lane; i < nc; i += kWave) S[i] = C[i] & ~1ull;
      }
      __syncthreads();
      bool done = false;
      if constexpr (DT == kF32) {
        // bfloat16 rows with an FP32 recheck, when its arrays fit as well
        if (a.base16 && 2u * pow2ceil_dev(nc) <= a.s_cap) {
          rechecked = rerank_bf16<D>(
              reinterpret_cast<const float*>(a.base), a.base16, a.norm16, S,
              nc, kq, reinterpret_cast<const float*>(q), oid, od, lane);
          done = true;
        }
      }
      if (!done) {
        // exact keys; each lane also keeps the smallest of its own
        uint64_t best = kInf;
        uint32_t at = kNone;
#pragma unroll 1
        for (uint32_t i = lane; i < nc; i += kWave) {
          const uint32_t id = key_id(S[i]);
          // the whole row in one round trip (the loop's registers are free)
          const uint64_t key =
              make_key(exact_dist<DT, D, true>(a.base, id, q, qq), id);
          S[i] = key;
          if (key < best) {
            best = key;
            at = i;
          }
        }
        __syncthreads();
        if (kq <= kWave)
          select_and_emit(S, nc, kq, best, at, oid, od, lane);
        else
          sort_and_emit(S, nc, kq, oid, od, lane);
        if (a.base16) rechecked = nc;
      }
    } else {
      // too many to sort in LDS: select in the candidate buffer itself
      for (uint32_t i = lane; i < nc; i += kWave) C[i] &= ~1ull;
      __threadfence();
      __syncthreads();
      if (nc > cmq) {
        global_select(C, nc, cmq, lane);
        nc = cmq;
      }
#pragma unroll 1
      for (uint32_t i = lane; i < nc; i += kWave) {
        const uint32_t id = key_id(C[i]);
        C[i] = make_key(exact_dist<DT, D, true>(a.base, id, q, qq), id);
      }
      __threadfence();
      __syncthreads();
      if (a.base16) rechecked = nc;
      global_select(C, nc, kq, lane);
      for (uint32_t i = lane; i < kq; i += kWave) {
        const uint64_t key = i < nc ? C[i] : kInf;
        oid[i] = key == kInf ? kNone : key_id(key);
        od[i] = key == kInf ? __uint_as_float(0x7F800000u) : key_dist(key);
      }
    }
    if (a.out_counters && a.base16 && lane == 0)
      a.out_counters[qi * 4 + 2] = rechecked;
    // a row of a mixed batch holds k_q results, then padding
    for (uint32_t i = kq + lane; i < a.k; i += kWave) {
      oid[i] = kNone;
      od[i] = __uint_as_float(0x7F800000u);
    }
    if (a.out_times && lane == 0) {
      a.out_times[qi * 2] = t_begin;
      a.out_times[qi * 2 + 1] = wall_clock64();
    }
    if constexpr (PHASES) {
      ph[6] = phase_clock() - tp;
      if (lane == 0)
        for (int p = 0; p < kPhases; ++p)
          a.out_phases[qi * kPhases + p] =
              (uint32_t)(ph[p] < 0xFFFFFFFFull ? ph[p] : 0xFFFFFFFFull);
    }
  }
}


// ---------------------------------------------------------------------------
// dispatch over the compiled (dtype, m, d/m) combinations
// ---------------------------------------------------------------------------
#define BANG_SHAPES(X) \
  X(16, 2) X(16, 4) X(16, 8) X(32, 2) X(32, 4) X(48, 2) X(64, 2)

template <template <int, int, int> class F, typename... Args>
hipError_t dispatch(int dt, uint32_t m, uint32_t ds, Args&&... args) {
#define BANG_CASE(MM, DD)                                                  \
  if (m == MM && ds == DD) {                                               \
    switch (dt) {                                                          \
      case kF32: return F<kF32, MM, DD>::run(args...);                     \
      case kU8: return F<kU8, MM, DD>::run(args...);                       \
      case kI8: return F<kI8, MM, DD>::run(args...);                       \
    }                                                                      \
  }
  BANG_SHAPES(BANG_CASE)
#undef BANG_CASE
  return hipErrorInvalidValue;
}

// Dynamic LDS above 64 KB per workgroup has to be enabled per kernel.
template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

template <typename K>
hipError_t occupancy_of(K kernel, size_t lds, int* per_cu) {
  // adc_codes addresses the table from LDS address 0, where the dynamic
  // LDS block starts only while the kernel declares no static LDS
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel));
  if (e != hipSuccess) return e;
  if (fa.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
  e = allow_lds(kernel, lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel, kWave,
                                                      lds);
}

}  // namespace

// The search variants, one per translation unit (search_variants.hip):
// v = host-resident adjacency (bit 0) | filter << 1 (none, Bloom, seen
// bitmap) | timed << 3; the timed variants exist for device-resident
// adjacency without the Bloom filter (v = 8, 12).  launch runs
// one search; occupancy gives the resident workgroups per CU at `lds` bytes
// of LDS and enables that LDS size for the kernel, so it precedes a launch.
#define BANG_VARIANT_DECL(V)                                                 \
  hipError_t search_launch_v##V(const SearchArgs& a, int dt, uint32_t m,     \
                                uint32_t ds, int table, uint32_t grid,       \
                                size_t lds, hipStream_t s);                  \
  hipError_t search_occupancy_v##V(int dt, uint32_t m, uint32_t ds,          \
                                   int table, size_t lds, int* per_cu);
BANG_VARIANT_DECL(0)
BANG_VARIANT_DECL(1)
BANG_VARIANT_DECL(2)
BANG_VARIANT_DECL(3)
BANG_VARIANT_DECL(4)
BANG_VARIANT_DECL(5)
BANG_VARIANT_DECL(8)
BANG_VARIANT_DECL(12)
#undef BANG_VARIANT_DECL

}  // namespace bang
