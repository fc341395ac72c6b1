// Device-side building blocks shared by the gfx950 kernels of the (T)
// library: operand traits per precision, the XOR-swizzled LDS layout, global
// address-space loads and stores, MFMA wrappers, the boxed W layout and the
// XCD-aware workgroup order.
#pragma once
#include "te_internal.h"

#include <stdint.h>

namespace te {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int WG = 256;

// ---------------------------------------------------------------- traits
template <Prec P> struct Tr;
// Output lane layout of the 16x16 MFMA blocks: lane l, register r holds
// column l%16 and row  (l/16) + 4r  for v_mfma_f64_16x16x4f64  (ROWQ = 1),
//                      4(l/16) + r  for the FP32 and BF16 forms (ROWQ = 4).
//
// LDS tiles are unpadded rows of KT elements. The 16-byte chunks of a row are
// XOR-swizzled: chunk c of row r is stored at chunk c ^ ((r / RP) % CR), with
// CR chunks per row. No padding is spent, which is what lets two (BF16x3,
// FP64) or three (FP32, BF16x2) workgroups share a CU.
//
// The LDS serves 128 bytes per clock (32 banks of 4 bytes: the W build's
// bank-conflict counter matches this model and not a 64-bank one), so a
// 16-byte-per-lane access runs in groups of 8 lanes. For the BF16 tiles (64
// bytes per row) RP is 2 rows: the 8 lanes of a fragment read take one chunk
// of 8 consecutive rows, which the swizzle puts in 8 distinct bank groups,
// and the chunk stores of a group cover whole rows: both conflict-free. The
// FP64 and FP32 fragments are one element per lane (16 rows at one k per
// 128 bytes, necessarily 2-way on 32 banks); there RP is 2 rows per 256
// bytes, which measured faster than conflict-free 16-byte reads that feed
// two or four k steps at once.
template <> struct Tr<Prec::F64> {
  using T = double; using Acc = d4; using Out = double;
  static constexpr int KT = 16, PAD = 0, NP = 1, KM = 4, ROWQ = 1;
  static constexpr bool SPLIT = false, SCALED = false;
};
template <> struct Tr<Prec::F32> {
  using T = float; using Acc = f4; using Out = float;
  static constexpr int KT = 32, PAD = 0, NP = 1, KM = 4, ROWQ = 4;
  static constexpr bool SPLIT = false, SCALED = false;
};
template <> struct Tr<Prec::BF16X3> {
  using T = uint16_t; using Acc = f4; using Out = float; using Frag = bf8;
  static constexpr int KT = 32, PAD = 0, NP = 3, KM = 32, ROWQ = 4;
  static constexpr bool SPLIT = true, SCALED = false;
};
template <> struct Tr<Prec::BF16X2> {
  using T = uint16_t; using Acc = f4; using Out = float; using Frag = bf8;
  static constexpr int KT = 32, PAD = 0, NP = 2, KM = 32, ROWQ = 4;
  static constexpr bool SPLIT = true, SCALED = false;
};
// FP16 parts of operands scaled by powers of two; the W build multiplies its
// result by WItem::scale.
template <> struct Tr<Prec::FP16X2> {
  using T = uint16_t; using Acc = f4; using Out = float; using Frag = h8;
  static constexpr int KT = 32, PAD = 0, NP = 2, KM = 32, ROWQ = 4;
  static constexpr bool SPLIT = true, SCALED = true;
};

template <typename TR> struct Swz {
  static constexpr int EC = 16 / sizeof(typename TR::T);            // elements per chunk
  static constexpr int CR = TR::KT / EC;                             // chunks per row
  static constexpr int RP = (TR::SPLIT ? 128 : 256) / (TR::KT * (int)sizeof(typename TR::T));
};
// Column of element k of LDS row r.
template <typename TR> __device__ inline int lcol(int r, int k) {
  using S = Swz<TR>;
  return ((((k / S::EC) ^ ((r / S::RP) % S::CR))) * S::EC) | (k % S::EC);
}
// Store eight consecutive elements (k0 % 8 == 0) of row r as swizzled chunks.
template <typename TR, typename T, typename CH>
__device__ inline void store_chunk(T *row, int r, int k0, const CH &c) {
  using S = Swz<TR>;
#pragma unroll
  for (int q = 0; q < CH::NQ; ++q)
    *reinterpret_cast<u32x4 *>(row + lcol<TR>(r, k0 + q * S::EC)) = c.q[q];
}

// Global-address-space views. Operand pointers reach the kernels through
// item structs in memory, so the compiler sees generic pointers and would
// emit FLAT accesses; FLAT loads count against the LDS counter too, which
// makes every wait for LDS fragments also wait for the next tile's prefetch.
template <typename T> using gptr = const __attribute__((address_space(1))) T *;
template <typename T> using gptr_w = __attribute__((address_space(1))) T *;
template <typename T> __device__ inline T gld(const T *p) { return *(gptr<T>)(p); }
template <typename T> __device__ inline void gst(T *p, T x) { *(gptr_w<T>)(p) = x; }

// Eight consecutive elements, moved as 16-byte words.
template <typename T> struct Chunk {
  static constexpr int NQ = sizeof(T) * 8 / 16;
  u32x4 q[NQ];
  __device__ T get(int e) const { return reinterpret_cast<const T *>(q)[e]; }
  __device__ void set(int e, T x) { reinterpret_cast<T *>(q)[e] = x; }
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < NQ; ++i) q[i] = u32x4{0u, 0u, 0u, 0u};
  }
  __device__ void load(const T *p) {
    gptr<u32x4> s = (gptr<u32x4>)(p);
#pragma unroll
    for (int i = 0; i < NQ; ++i) q[i] = s[i];
  }
  // from a base shared by the wave plus a per-lane 32-bit byte offset (lets
  // the compiler use a scalar base register and no 64-bit address add)
  __device__ void load_at(const T *base, uint32_t byte_off) {
    gptr<u32x4> s = (gptr<u32x4>)(reinterpret_cast<const char *>(base) + byte_off);
#pragma unroll
    for (int i = 0; i < NQ; ++i) q[i] = s[i];
  }
};

// Choice between two values. A conditional over two lvalues (array elements,
// struct members) is one over their addresses, which can send the whole
// array or struct to scratch memory; this one is over the loaded values.
template <typename T> __device__ inline T pick(bool c, T a, T b) { return c ? a : b; }

__device__ inline d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4 mma(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f4 mma(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ inline long box_off(int a, int b, int c, int nT) {
  return ((((long)(a >> 3) * nT + (b >> 3)) * nT + (c >> 3)) << 9) + ((a & 7) << 6) +
         ((b & 7) << 3) + (c & 7);
}

// Logical tile id such that consecutive ids share an XCD (workgroups are
// dispatched round-robin over the 8 XCDs of the chip).
__device__ inline long xcd_remap(long bid, long total) {
  long per = total >> 3, rem = total & 7;
  long x = bid & 7, q = bid >> 3;
  return x * per + (x < rem ? x : rem) + q;
}

}  // namespace
}  // namespace te
