// pinn_device.h -- device code shared by the gfx950 kernels of the fused PINN residual +
// gradient step: operand formats and matrix-core products, LDS tile layouts, activation
// and PDE-residual jets, and the forward / layer-backward bodies that several kernels use.
// Included by the kernel translation units only.
#pragma once

// Data model.  Every point carries 4 jet channels: value, first derivatives in the inputs
// (d_in of them) and, when the PDE needs it, the Laplacian over the inputs in lap_mask;
// unused channels stay zero.  A tile of P points is a (4P x width) matrix whose rows are
// "cp" = 4 * point + channel, so one linear layer (Sec. 2.2, z = W a + b) is the matrix
// product Z = A W^T over all channels at once, with the bias added on the value channel
// only.  The products run on the matrix cores:
//   FP32    v_mfma_f32_16x16x4_f32, 8 per 32-wide reduction chunk;
//   BF16X3  v_mfma_f32_16x16x32_bf16 three times per chunk: hi*hi + hi*lo + lo*hi with
//           x = hi + lo, hi = bf16(x), lo = bf16(x - hi).
// An operand fragment is 32 bytes per lane for both precisions (8 FP32, or 8 hi + 8 lo
// BF16), so tiles in LDS and weight fragments in memory have one layout for both.
//
// Accumulator layout of a 16x16 product block (verified on the device): lane l holds
// column l % 16 and rows 4 * (l / 16) + r, r = 0..3.  With M = cp rows, the 4 registers
// of a lane are the 4 channels of one (point, neuron): the activation jet update is
// lane-local.
//
// Kernels (one translation unit each group, so that they compile in parallel):
//   k_misc.hip      k_prepare (in one launch: residual and supervision points gathered into
//                   one padded buffer, effective weights W = diag(exp s) V, Sec. 2.6.2, and
//                   operand fragments), k_grad0 (identity-embedding first layer's weight
//                   gradient), k_reduce_all (fixed-order FP64 reductions of every layer's
//                   per-work-group partial sums and of the loss terms, one launch), the other
//                   k_reduce_* kernels;
//   k_forward.hip   per tile: embedding jets, hidden layers, output layer, residual, loss
//                   partial sums, residual adjoint seed and the output layer's backward;
//                   stores the pre-activation jets of the hidden layers the backward reads;
//   k_backward.hip  one linear layer's backward over a range of sub-tiles: weight gradient
//                   (kept in registers over the range), adjoint of the layer input and the
//                   activation adjoint;
//   k_batched.hip   many independent networks in one persistent launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pinn_internal.h"

namespace pinn {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) float f4;

struct Raw {
  uint4 a, b;
};

__device__ __forceinline__ float4 to_float4(f4 v) { return make_float4(v.x, v.y, v.z, v.w); }
__device__ __forceinline__ f4 to_f4(float4 v) { return f4{v.x, v.y, v.z, v.w}; }

// ------------------------------------------------------------------ precision policy

template <int PREC>
struct Prec;

template <>
struct Prec<kFP32> {
  static __device__ __forceinline__ void mma(f4& acc, const Raw& x, const Raw& y) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.a.x), __uint_as_float(y.a.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.a.y), __uint_as_float(y.a.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.a.z), __uint_as_float(y.a.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.a.w), __uint_as_float(y.a.w), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.b.x), __uint_as_float(y.b.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.b.y), __uint_as_float(y.b.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.b.z), __uint_as_float(y.b.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x.b.w), __uint_as_float(y.b.w), acc, 0, 0, 0);
  }
  // acc[i][c] += a[c] * b[i] for a whole register tile; the loops run over independent
  // accumulators innermost so that consecutive products never wait on each other.  The
  // order of the eight partial products into each accumulator is that of mma().
  template <int NB, int CB>
  static __device__ __forceinline__ void mma_tile(f4 (&acc)[NB][CB], const Raw (&a)[CB], const Raw (&b)[NB]) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const uint32_t x = j < 4 ? (&a[c].a.x)[j] : (&a[c].b.x)[j - 4];
          const uint32_t y = j < 4 ? (&b[i].a.x)[j] : (&b[i].b.x)[j - 4];
          acc[i][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x), __uint_as_float(y), acc[i][c], 0, 0, 0);
        }
  }
  static __device__ __forceinline__ Raw make(const float (&f)[8]) {
    Raw r;
    r.a = make_uint4(__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]), __float_as_uint(f[3]));
    r.b = make_uint4(__float_as_uint(f[4]), __float_as_uint(f[5]), __float_as_uint(f[6]), __float_as_uint(f[7]));
    return r;
  }
  // one element at position pos (0..7) of a 32-byte unit
  static __device__ __forceinline__ void put(char* unit, int pos, float x) {
    reinterpret_cast<float*>(unit)[pos] = x;
  }
  // four consecutive elements at pos0 (0 or 4)
  static __device__ __forceinline__ void put4(char* unit, int pos0, f4 x) {
    *reinterpret_cast<float4*>(unit + 4 * pos0) = to_float4(x);
  }
  // two consecutive elements at an even position
  static __device__ __forceinline__ void put2(char* unit, int pos, float x, float y) {
    *reinterpret_cast<float2*>(unit + 4 * pos) = make_float2(x, y);
  }
};

__device__ __forceinline__ __bf16 bf16_rne(float x) { return (__bf16)x; }

typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(2))) _Float16 f16x2;

// The 16-bit format of a split precision: conversion of two values into hi and lo parts
// (x = hi + lo, hi = rn(x), lo = rn(x - hi), round to nearest even) and one matrix-core
// product of 8-element operand halves.
template <int PREC>
struct Half;

template <>
struct Half<kBF16X3> {
  // one packed conversion per part, the hi parts widened back by shifts
  static __device__ __forceinline__ void split2(float x, float y, uint32_t& h, uint32_t& l) {
    bf16x2 hv;
    hv[0] = bf16_rne(x);
    hv[1] = bf16_rne(y);
    h = __builtin_bit_cast(uint32_t, hv);
    const float xh = __uint_as_float(h << 16), yh = __uint_as_float(h & 0xffff0000u);
    bf16x2 lv;
    lv[0] = bf16_rne(x - xh);
    lv[1] = bf16_rne(y - yh);
    l = __builtin_bit_cast(uint32_t, lv);
  }
  static __device__ __forceinline__ f4 mfma(const uint4& a, const uint4& b, f4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc,
                                                   0, 0, 0);
  }
};

// IEEE half: 11 significant bits per part, so hi + lo carries 22 (bf16: 16) -- the
// representation error of an operand drops from 2^-16 to 2^-22 relative, at the same
// matrix-core rate.  The range is that of half precision: parts below 2^-14 are subnormal
// (absolute resolution 2^-24), magnitudes from 65520 up overflow.  Adjoints are therefore
// scaled by a power of two before they are split (adj_scale).
template <>
struct Half<kFP16X3> {
  static __device__ __forceinline__ void split2(float x, float y, uint32_t& h, uint32_t& l) {
    f16x2 hv;
    hv[0] = (_Float16)x;
    hv[1] = (_Float16)y;
    h = __builtin_bit_cast(uint32_t, hv);
    f16x2 lv;
    lv[0] = (_Float16)(x - (float)hv[0]);
    lv[1] = (_Float16)(y - (float)hv[1]);
    l = __builtin_bit_cast(uint32_t, lv);
  }
  static __device__ __forceinline__ f4 mfma(const uint4& a, const uint4& b, f4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), acc, 0,
                                                  0, 0);
  }
};

// The split product: a Raw fragment is 8 hi parts (a) then 8 lo parts (b).
template <int PREC>
struct PrecSplit {
  using H = Half<PREC>;
  static __device__ __forceinline__ void mma(f4& acc, const Raw& x, const Raw& y) {
    acc = H::mfma(x.b, y.a, acc);
    acc = H::mfma(x.a, y.b, acc);
    acc = H::mfma(x.a, y.a, acc);
  }
  // Register-tile form of mma(): each of the three products in turn over all
  // accumulators, same per-accumulator order as mma().
  template <int NB, int CB>
  static __device__ __forceinline__ void mma_tile(f4 (&acc)[NB][CB], const Raw (&a)[CB], const Raw (&b)[NB]) {
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int i = 0; i < NB; ++i) acc[i][c] = H::mfma(a[c].b, b[i].a, acc[i][c]);
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int i = 0; i < NB; ++i) acc[i][c] = H::mfma(a[c].a, b[i].b, acc[i][c]);
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int i = 0; i < NB; ++i) acc[i][c] = H::mfma(a[c].a, b[i].a, acc[i][c]);
  }
  static __device__ __forceinline__ Raw make(const float (&f)[8]) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) H::split2(f[2 * j], f[2 * j + 1], h[j], l[j]);
    Raw r;
    r.a = make_uint4(h[0], h[1], h[2], h[3]);
    r.b = make_uint4(l[0], l[1], l[2], l[3]);
    return r;
  }
  static __device__ __forceinline__ void put2(char* unit, int pos, float x, float y) {
    uint32_t h, l;
    H::split2(x, y, h, l);
    *reinterpret_cast<uint32_t*>(unit + 2 * pos) = h;
    *reinterpret_cast<uint32_t*>(unit + 16 + 2 * pos) = l;
  }
  static __device__ __forceinline__ void put4(char* unit, int pos0, f4 x) {
    uint32_t h0, l0, h1, l1;
    H::split2(x[0], x[1], h0, l0);
    H::split2(x[2], x[3], h1, l1);
    *reinterpret_cast<uint2*>(unit + 2 * pos0) = make_uint2(h0, h1);
    *reinterpret_cast<uint2*>(unit + 16 + 2 * pos0) = make_uint2(l0, l1);
  }
};

template <>
struct Prec<kBF16X3> : PrecSplit<kBF16X3> {};
template <>
struct Prec<kFP16X3> : PrecSplit<kFP16X3> {};

// Power-of-two scale of an adjoint before it is split into 16-bit parts, from the largest
// magnitude `amax` (FP32 bits) of that adjoint: FP16X3 maps the largest magnitude into
// [2^14, 2^15) (half precision tops out at 65504), the other precisions use 1.  Scaling by
// a power of two is exact, and the product's result is scaled back by the reciprocal.
template <int PREC>
__device__ __forceinline__ float adj_scale(unsigned int amax) {
  if constexpr (PREC != kFP16X3) {
    return 1.0f;
  } else {
    const int e = (int)((amax >> 23) & 0xffu);
    if (amax == 0u || e == 0xff) return 1.0f;  // all zero, or not finite
    return __builtin_ldexpf(1.0f, 14 - (e - 127));
  }
}

// Largest magnitude of the 4 channels of a jet.
__device__ __forceinline__ float jet_absmax(f4 v) {
  return fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w)));
}

// v * s for the precision that scales adjoints, v otherwise.
template <int PREC>
__device__ __forceinline__ f4 ascale(f4 v, float s) {
  if constexpr (PREC == kFP16X3) return v * s;
  return v;
}
template <int PREC>
__device__ __forceinline__ float ascale(float v, float s) {
  if constexpr (PREC == kFP16X3) return v * s;
  return v;
}

// Combine a per-lane largest magnitude over the wave and into *word (FP32 bits of a
// non-negative value compare as unsigned integers).
__device__ __forceinline__ void amax_publish(float m, unsigned int* word) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(word, __float_as_uint(m));
}

// Value of lane l ^ 1 (a data-parallel-primitive lane swap within each pair of lanes).
__device__ __forceinline__ float swap_pair(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}

// Write the 4 channels of column n (rows base, base + rs, ... of an R-layout tile, unit of
// column n already applied).  Lanes l and l ^ 1 hold neighbouring columns n (even) and
// n + 1; after one exchange the even lane writes rows 0 and 1 and the odd lane rows 2 and
// 3, two columns per write: half the LDS writes of one column per write.  Both lanes of
// every pair must be active.
template <int PREC>
__device__ __forceinline__ void put_rows(char* base, int rs, int n, f4 a) {
  const bool odd = n & 1;
  const float r0 = swap_pair(odd ? a[0] : a[2]);
  const float r1 = swap_pair(odd ? a[1] : a[3]);
  const int row = odd ? 2 : 0, pos = n & 6;
  Prec<PREC>::put2(base + (size_t)row * rs, pos, odd ? r0 : a[0], odd ? a[2] : r0);
  Prec<PREC>::put2(base + (size_t)(row + 1) * rs, pos, odd ? r1 : a[1], odd ? a[3] : r1);
}

__device__ __forceinline__ Raw lds_unit(const char* base, int row, int unit, int stride) {
  const uint4* p = reinterpret_cast<const uint4*>(base + (size_t)row * stride + unit * 32);
  Raw r;
  r.a = p[0];
  r.b = p[1];
  return r;
}

// Row strides of the two LDS tile layouts (bytes).  "R": rows cp, units over neurons.
// "Q": rows neurons, units over cp in the order of the product accumulators.
__host__ __device__ constexpr int r_stride(int width) { return width * 4 + 16; }
__host__ __device__ constexpr int q_stride(int cp) { return cp * 4 + 16; }

// ------------------------------------------------------------------ A-operand jet tiles
// A tile holds the jets of P points x K neurons as the A operand of a product (rows
// cp = 4 point + channel, reduction over neurons).  `ld` is the layout's leading size.
//   FP32   "R" layout: rows cp (ld = row stride in bytes), 32-byte units of 8 neurons; a
//          fragment is one unit.
//   BF16X3 "T" layout: the 4 channels of a (point, neuron) are 4 consecutive bf16, hi and lo
//          parts in two 1 KiB cells per 4 points x 32 neurons, cells ordered by neuron
//          chunk then point group (ld = point groups of 4 in the tile).
//          Stored with one 8-byte write per part; a fragment is 4 transposing LDS reads
//          (ds_read_b64_tr_b16: within each 16-lane group, lane 4q + j receives element j of
//          the 8 bytes read by lanes q, q + 4, q + 8 and q + 12).  The in-cell swizzle
//          keeps both the writes of an accumulator block and the fragment reads free of
//          bank conflicts per half wave.
template <int PREC>
struct Tile;

template <>
struct Tile<kFP32> {
  static __device__ __forceinline__ int ld(int kmax, int P) { return r_stride(kmax); }
  static __device__ __forceinline__ void put(char* X, int ld, int p, int n, f4 a) {
    put_rows<kFP32>(X + (size_t)(4 * p) * ld + (n >> 3) * 32, ld, n, a);
  }
  static __device__ __forceinline__ Raw load(const char* X, int ld, int cb, int kc, int lane) {
    return lds_unit(X, 16 * cb + (lane & 15), 4 * kc + (lane >> 4), ld);
  }
};

// Byte offset of (point p mod 4, neuron n mod 32) inside a T-layout cell.
__device__ __forceinline__ int t_cell_off(int p, int n) {
  const int p0 = p & 1, p1 = (p >> 1) & 1;
  const int n0 = n & 1, n1 = (n >> 1) & 1, n2 = (n >> 2) & 1, n3 = (n >> 3) & 1, n4 = (n >> 4) & 1;
  const int slot = p0 | (n0 << 1) | (n1 << 2) | (n3 << 3) | ((n2 ^ p1) << 4);
  return ((n4 << 1) | p1) * 256 + slot * 8;
}

typedef short v4s __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint2 lds_tr16(const char* p) {
  const v4s v = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) v4s*)(const_cast<char*>(p)));
  return __builtin_bit_cast(uint2, v);
}

// LDS byte address of a pointer into the work-group's LDS, masked to the 18 bits an LDS
// address has: with the high bits known to be zero the compiler folds constant offsets
// added to it into the immediate offset of the LDS instruction instead of adding them per
// access.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)p & 0x3FFFFu;
}
__device__ __forceinline__ uint2 lds_tr16_at(uint32_t a) {
  const v4s v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) v4s*)(uintptr_t)a);
  return __builtin_bit_cast(uint2, v);
}

template <int PREC>
struct TileT {
  static __device__ __forceinline__ int ld(int kmax, int P) { return P >> 2; }
  static __device__ __forceinline__ char* cell(char* X, int ld, int pg, int nc) {
    return X + (size_t)(nc * ld + pg) * 2048;
  }
  static __device__ __forceinline__ void put(char* X, int ld, int p, int n, f4 a) {
    uint32_t h0, l0, h1, l1;
    Half<PREC>::split2(a[0], a[1], h0, l0);
    Half<PREC>::split2(a[2], a[3], h1, l1);
    char* q = cell(X, ld, p >> 2, n >> 5) + t_cell_off(p, n);
    *reinterpret_cast<uint2*>(q) = make_uint2(h0, h1);
    *reinterpret_cast<uint2*>(q + 1024) = make_uint2(l0, l1);
  }
  static __device__ __forceinline__ Raw load(const char* X, int ld, int cb, int kc, int lane) {
    const int g = lane >> 4, s = lane & 15;
    const uint32_t c = (uint32_t)(kc * ld + cb) * 2048;
    const uint32_t x0 = (lds_addr(X) + t_cell_off(s, 8 * g + (s >> 2))) & 0x3FFFFu;
    const uint32_t x1 = (lds_addr(X) + t_cell_off(s, 8 * g + 4 + (s >> 2))) & 0x3FFFFu;
    const uint2 h0 = lds_tr16_at(x0 + c), h1 = lds_tr16_at(x1 + c);
    const uint2 l0 = lds_tr16_at(x0 + c + 1024), l1 = lds_tr16_at(x1 + c + 1024);
    Raw r;
    r.a = make_uint4(h0.x, h0.y, h1.x, h1.y);
    r.b = make_uint4(l0.x, l0.y, l1.x, l1.y);
    return r;
  }
};

template <>
struct Tile<kBF16X3> : TileT<kBF16X3> {};
template <>
struct Tile<kFP16X3> : TileT<kFP16X3> {};

__device__ __forceinline__ Raw glob_frag(const char* frags, int blk, int chunk, int nchunk, int lane) {
  const uint4* p = reinterpret_cast<const uint4*>(frags + (((size_t)blk * nchunk + chunk) * 64 + lane) * 32);
  Raw r;
  r.a = p[0];
  r.b = p[1];
  return r;
}


// Q-layout position of a cp row inside its 32-row chunk: the accumulator of cp block cb,
// lane group g, register r sits at 8 g + 4 (cb % 2) + r.
__device__ __forceinline__ void q_pos(int cb, int g, int& unit, int& pos0) {
  unit = 4 * (cb >> 1) + g;
  pos0 = 4 * (cb & 1);
}

// Fragment-major jet buffer: fragment (cb, nb) is 64 lanes x 4 floats, lane l holds
// neuron 16 nb + l % 16 of point 4 cb + l / 16, channels 0..3.
__device__ __forceinline__ float4* jet_frag(float* buf, int64_t cb, int nb, int nbs, int lane) {
  return reinterpret_cast<float4*>(buf) + ((cb * nbs + nb) * 64 + lane);
}

// Jet-fragment stores of one tile through a buffer resource over the tile's bytes: a store
// switched off by a wave-uniform condition goes to an offset past the end, which the
// hardware drops, instead of behind a branch.  The number of vector-memory operations a wave
// has issued then does not depend on the condition, so later waits for loads issued before
// these stores can leave the stores in flight.
// Cache-policy operand of the buffer intrinsics for a non-temporal (streaming) access.
constexpr int kNonTemporal = 2;

struct FragStore {
  __amdgpu_buffer_rsrc_t r;
  int nbs;
  __device__ __forceinline__ FragStore(float* buf, int64_t cb0, int ncb, int nbs_) : nbs(nbs_) {
    r = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<float4*>(buf) + cb0 * nbs_ * 64, (short)0,
                                          ncb * nbs_ * 1024, 0x00020000);
  }
  // cp block cb (relative to cb0), neuron block nb, stored only when ok
  __device__ __forceinline__ void put(int cb, int nb, int lane, f4 v, bool ok) const {
    typedef __attribute__((ext_vector_type(4))) unsigned u4v;
    // the condition goes through a register the compiler cannot see into, so that it selects
    // the offset instead of duplicating the code around a branch
    int okv = ok;
    asm volatile("" : "+v"(okv));
    const unsigned off = okv ? (unsigned)(((cb * nbs + nb) * 64 + lane) * 16) : 0x80000000u;
    // non-temporal: the backward reads the stash long after, so it should not displace
    // what this kernel re-reads from cache (the weight fragments)
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, v), r, off, 0, kNonTemporal);
  }
};

// acc[i][c] += A(cp block cb0 + c) * W(block blk[i])^T over all reduction chunks: the A
// operand comes from a jet tile in LDS (Tile<PREC>), the B operand from fragment-major
// weights.
// Every block index must be valid (callers clamp them; results of clamped duplicates are
// discarded), so the loop body has no branches and the products of one chunk issue back
// to back over independent accumulators.
// PRE: the weight fragments of chunks 0 and 1 (chunk 0 again when there is one chunk) come
// in pre0 / pre1, loaded by the caller before its own stores, so that waiting for them does
// not wait for those stores (vector-memory counters complete in issue order).
template <int PREC, int NB, int CB, int CGMAX = 8, bool PREFETCH = false, bool PRE = false>
__device__ __forceinline__ void gemm_tile(f4 (&acc)[NB][CB], const char* X, int ld, int cb0,
                                          const char* frags, int kchunks, const int (&blk)[NB], int lane,
                                          const Raw (&pre0)[NB], const Raw (&pre1)[NB]) {
  static_assert(!PRE || PREFETCH, "preloaded chunks need the prefetching loop");
  const char* fb[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) fb[i] = frags + ((size_t)blk[i] * kchunks * 64 + lane) * 32;
  constexpr int CG = CB > CGMAX ? CGMAX : CB;  // A fragments live at a time
  static_assert(CB % CG == 0, "cp blocks per wave");
  auto load_b = [&](Raw (&b)[NB], int kc) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const uint4* p = reinterpret_cast<const uint4*>(fb[i] + (size_t)kc * 2048);
      b[i].a = p[0];
      b[i].b = p[1];
    }
  };
  Raw bw[NB];
  if (PRE) {
#pragma unroll
    for (int i = 0; i < NB; ++i) bw[i] = pre0[i];
  } else if (PREFETCH) {
    load_b(bw, 0);  // weight fragments of chunk kc + 1 load while chunk kc multiplies
  }
  for (int kc = 0; kc < kchunks; ++kc) {
    Raw bn[NB];
    if (PRE && kc == 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) bn[i] = pre1[i];
    } else if (PREFETCH) {
      load_b(bn, kc + 1 < kchunks ? kc + 1 : kc);
    } else {
      load_b(bw, kc);
    }
#pragma unroll
    for (int c0 = 0; c0 < CB; c0 += CG) {
      Raw a[CG];
#pragma unroll
      for (int c = 0; c < CG; ++c) a[c] = Tile<PREC>::load(X, ld, cb0 + c0 + c, kc, lane);
      f4 (&part)[NB][CB] = acc;
      f4 sub[NB][CG];
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int c = 0; c < CG; ++c) sub[i][c] = part[i][c0 + c];
      Prec<PREC>::template mma_tile<NB, CG>(sub, a, bw);
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int c = 0; c < CG; ++c) part[i][c0 + c] = sub[i][c];
    }
    if (PREFETCH) {
#pragma unroll
      for (int i = 0; i < NB; ++i) bw[i] = bn[i];
    }
  }
}

template <int PREC, int NB, int CB, int CGMAX = 8, bool PREFETCH = false>
__device__ __forceinline__ void gemm_tile(f4 (&acc)[NB][CB], const char* X, int ld, int cb0,
                                          const char* frags, int kchunks, const int (&blk)[NB], int lane) {
  Raw none[NB];
  gemm_tile<PREC, NB, CB, CGMAX, PREFETCH, false>(acc, X, ld, cb0, frags, kchunks, blk, lane, none, none);
}

// Weight fragments of chunks 0 and 1 of blocks blk (chunk 0 twice when there is one chunk).
template <int NB>
__device__ __forceinline__ void load_first_chunks(Raw (&b0)[NB], Raw (&b1)[NB], const char* frags, int kchunks,
                                                  const int (&blk)[NB], int lane) {
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    b0[i] = glob_frag(frags, blk[i], 0, kchunks, lane);
    b1[i] = glob_frag(frags, blk[i], kchunks > 1 ? 1 : 0, kchunks, lane);
  }
}

// ------------------------------------------------------------------ activation

// tanh z = 1 - 2 / (exp(2|z|) + 1), sign of z; the hardware base-2 exponential and
// reciprocal (absolute error about 1e-7, far below the FP32 tolerance of the path).
__device__ __forceinline__ float tanh_fast(float z) {
  const float e = __builtin_amdgcn_exp2f(fabsf(z) * 2.885390043258667f);  // exp(2|z|)
  const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
  return copysignf(t, z);
}

// sin and cos: Cody-Waite reduction by 2 pi with a two-part constant (each step one fused
// multiply-add, so the reduced argument is accurate to FP32 rounding), then the hardware
// sine and cosine, which take their argument in revolutions.
__device__ __forceinline__ void sincos_fast(float x, float& s, float& c) {
  const float k = rintf(x * 0.15915493667125702f);
  float r = fmaf(-k, 6.2831854820251465f, x);
  r = fmaf(-k, -1.7484555314695172e-07f, r);
  const float u = r * 0.15915493667125702f;
  s = __builtin_amdgcn_sinf(u);
  c = __builtin_amdgcn_cosf(u);
}

template <int ACT>
__device__ __forceinline__ void act_eval(float z, float w0, float& s0, float& s1, float& s2, float& s3) {
  if ((ACT & 1) == kTanh) {
    const float t = tanh_fast(z);
    const float d = 1.0f - t * t;
    s0 = t;
    s1 = d;
    s2 = -2.0f * t * d;
    s3 = d * (6.0f * t * t - 2.0f);
  } else {
    float sn, cs;
    sincos_fast(w0 * z, sn, cs);
    s0 = sn;
    s1 = w0 * cs;
    s2 = -w0 * w0 * sn;
    s3 = -w0 * w0 * w0 * cs;
  }
}

// Weights of the first-derivative channels in the Laplacian channel (channel 3): 1 for the
// inputs in the Laplacian set, 0 otherwise; both 0 when channel 3 is a plain derivative
// (three inputs) or unused.  Wave-uniform.
__device__ __forceinline__ void lap_weights(const NetDev& net, float& w1, float& w2) {
  const bool lap = net.lapch == 3;
  w1 = lap && (net.lap_mask & 1) ? 1.0f : 0.0f;
  w2 = lap && (net.lap_mask & 2) ? 1.0f : 0.0f;
}

// Jet of sigma(z): value s0, first derivatives s1 dz, and in channel 3 either the
// derivative s1 dz_3 (LAP false: three inputs, or an unused channel) or the Laplacian
// s2 sum_S (dz_k)^2 + s1 Lap z (LAP true; w1, w2 select the inputs in S).
template <bool LAP>
__device__ __forceinline__ f4 jet_act(f4 z, float s0, float s1, float s2, float w1, float w2) {
  f4 a;
  a.x = s0;
  a.y = s1 * z.y;
  a.z = s1 * z.z;
  a.w = s1 * z.w;
  if (LAP) a.w = fmaf(s2, w1 * z.y * z.y + w2 * z.z * z.z, a.w);
  return a;
}

// Transpose of jet_act: adjoints of z given the adjoints abar of the activation jet.
template <bool LAP>
__device__ __forceinline__ f4 jet_act_adj(f4 z, f4 ab, float s1, float s2, float s3, float w1, float w2) {
  f4 zb;
  zb.y = ab.y * s1;
  zb.z = ab.z * s1;
  zb.w = ab.w * s1;
  zb.x = ab.x * s1 + s2 * (ab.y * z.y + ab.z * z.z + ab.w * z.w);
  if (LAP) {
    const float t = 2.0f * ab.w * s2;
    zb.x = fmaf(ab.w * s3, w1 * z.y * z.y + w2 * z.z * z.z, zb.x);
    zb.y = fmaf(t * w1, z.y, zb.y);
    zb.z = fmaf(t * w2, z.z, zb.z);
  }
  return zb;
}

// ------------------------------------------------------------------ PDE residuals

// Output jets y[o][c] (c: 0 value, 1.. derivatives, lapch Laplacian) -> residuals r and,
// with the seed scale g_c = 2 lambda_c / N, the output-jet adjoint yb[o][c].
template <typename T, typename C>
__device__ __forceinline__ void residual_point_t(int pde_id, const C* coef, const C* g, const T (&y)[kMaxOut][4],
                                                 T (&r)[kMaxOut], T (&yb)[kMaxOut][4]) {
#pragma unroll
  for (int o = 0; o < kMaxOut; ++o) {
    r[o] = T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) yb[o][c] = T(0);
  }
  switch (pde_id) {
    case kBurgers: {  // (x, t): u_t + u u_x - nu u_xx
      const T nu = (T)coef[0];
      const T u = y[0][0], ux = y[0][1], ut = y[0][2], uxx = y[0][3];
      r[0] = ut + u * ux - nu * uxx;
      const T b = (T)g[0] * r[0];
      yb[0][0] = b * ux;
      yb[0][1] = b * u;
      yb[0][2] = b;
      yb[0][3] = -b * nu;
      break;
    }
    case kEuler1D: {  // (x, t) -> (rho, u, p), conservative form expanded by the product rule
      const T k = T(1) / ((T)coef[0] - T(1));
      const T rho = y[0][0], rx = y[0][1], rt = y[0][2];
      const T u = y[1][0], ux = y[1][1], ut = y[1][2];
      const T p = y[2][0], px = y[2][1], pt = y[2][2];
      const T uu = u * u;
      r[0] = rt + u * rx + rho * ux;
      r[1] = u * rt + rho * ut + uu * rx + T(2) * rho * u * ux + px;
      r[2] = k * pt + T(0.5) * uu * rt + rho * u * ut + (k + T(1)) * (u * px + p * ux) +
             T(0.5) * uu * u * rx + T(1.5) * rho * uu * ux;
      const T b0 = (T)g[0] * r[0], b1 = (T)g[1] * r[1], b2 = (T)g[2] * r[2];
      yb[0][0] = b0 * ux + b1 * (ut + T(2) * u * ux) + b2 * (u * ut + T(1.5) * uu * ux);
      yb[0][1] = b0 * u + b1 * uu + b2 * T(0.5) * uu * u;
      yb[0][2] = b0 + b1 * u + b2 * T(0.5) * uu;
      yb[1][0] = b0 * rx + b1 * (rt + T(2) * u * rx + T(2) * rho * ux) +
                 b2 * (u * rt + rho * ut + (k + T(1)) * px + T(1.5) * uu * rx + T(3) * rho * u * ux);
      yb[1][1] = b0 * rho + b1 * T(2) * rho * u + b2 * ((k + T(1)) * p + T(1.5) * rho * uu);
      yb[1][2] = b1 * rho + b2 * rho * u;
      yb[2][0] = b2 * (k + T(1)) * ux;
      yb[2][1] = b1 + b2 * (k + T(1)) * u;
      yb[2][2] = b2 * k;
      break;
    }
    case kNS2D: {  // (x, y) -> (u, v, p), steady incompressible, 1/Re viscosity
      const T iRe = T(1) / (T)coef[0];
      const T u = y[0][0], ux = y[0][1], uy = y[0][2], lu = y[0][3];
      const T v = y[1][0], vx = y[1][1], vy = y[1][2], lv = y[1][3];
      const T px = y[2][1], py = y[2][2];
      r[0] = ux + vy;
      r[1] = u * ux + v * uy + px - iRe * lu;
      r[2] = u * vx + v * vy + py - iRe * lv;
      const T b0 = (T)g[0] * r[0], b1 = (T)g[1] * r[1], b2 = (T)g[2] * r[2];
      yb[0][0] = b1 * ux + b2 * vx;
      yb[0][1] = b0 + b1 * u;
      yb[0][2] = b1 * v;
      yb[0][3] = -b1 * iRe;
      yb[1][0] = b1 * uy + b2 * vy;
      yb[1][1] = b2 * u;
      yb[1][2] = b0 + b2 * v;
      yb[1][3] = -b2 * iRe;
      yb[2][1] = b1;
      yb[2][2] = b2;
      break;
    }
    case kMaxwell: {  // (x, y, t) -> (E_z, H_x, H_y)
      const T ie = T(1) / (T)coef[0], im = T(1) / (T)coef[1];
      const T ezx = y[0][1], ezy = y[0][2], ezt = y[0][3];
      const T hxy = y[1][2], hxt = y[1][3];
      const T hyx = y[2][1], hyt = y[2][3];
      r[0] = ezt - ie * (hyx - hxy);
      r[1] = hxt + im * ezy;
      r[2] = hyt - im * ezx;
      const T b0 = (T)g[0] * r[0], b1 = (T)g[1] * r[1], b2 = (T)g[2] * r[2];
      yb[0][3] = b0;
      yb[2][1] = -b0 * ie;
      yb[1][2] = b0 * ie;
      yb[1][3] = b1;
      yb[0][2] = b1 * im;
      yb[2][3] = b2;
      yb[0][1] = -b2 * im;
      break;
    }
    case kAdvection: {  // (x, t): u_t + c u_x
      const T c = (T)coef[0];
      r[0] = y[0][2] + c * y[0][1];
      const T b = (T)g[0] * r[0];
      yb[0][1] = b * c;
      yb[0][2] = b;
      break;
    }
    case kAllenCahn: {  // (x, t): u_t - D u_xx + k u^3 - k u
      const T D = (T)coef[0], k = (T)coef[1];
      const T u = y[0][0], ut = y[0][2], uxx = y[0][3];
      r[0] = ut - D * uxx + k * u * u * u - k * u;
      const T b = (T)g[0] * r[0];
      yb[0][0] = b * k * (T(3) * u * u - T(1));
      yb[0][2] = b;
      yb[0][3] = -b * D;
      break;
    }
    case kEuler2D: {  // (x, y, t) -> (rho, u, v, p), conservative form expanded by the product rule
      // e = rho E = k p + rho q / 2 with q = u^2 + v^2 and k = 1 / (gamma - 1); the energy
      // flux is (u, v) h with h = e + p, whose derivatives hx, hy enter the last equation
      const T k = T(1) / ((T)coef[0] - T(1));
      const T rho = y[0][0], rx = y[0][1], ry = y[0][2], rt = y[0][3];
      const T u = y[1][0], ux = y[1][1], uy = y[1][2], ut = y[1][3];
      const T v = y[2][0], vx = y[2][1], vy = y[2][2], vt = y[2][3];
      const T p = y[3][0], px = y[3][1], py = y[3][2], pt = y[3][3];
      const T k1 = k + T(1), q = u * u + v * v, hq = T(0.5) * q;
      const T h = k1 * p + rho * hq;
      const T hx = k1 * px + hq * rx + rho * (u * ux + v * vx);
      const T hy = k1 * py + hq * ry + rho * (u * uy + v * vy);
      const T et = k * pt + hq * rt + rho * (u * ut + v * vt);
      // material derivative of rho and the divergence of (u, v)
      const T dr = rt + u * rx + v * ry, dv = ux + vy;
      const T du = ut + u * ux + v * uy, dvv = vt + u * vx + v * vy;
      r[0] = dr + rho * dv;
      r[1] = u * r[0] + rho * du + px;
      r[2] = v * r[0] + rho * dvv + py;
      r[3] = et + dv * h + u * hx + v * hy;
      const T b0 = (T)g[0] * r[0], b1 = (T)g[1] * r[1], b2 = (T)g[2] * r[2], b3 = (T)g[3] * r[3];
      // r1 and r2 reach the jets through r0 as well: its total weight c0
      const T c0 = b0 + b1 * u + b2 * v;
      // adjoints of the energy intermediates
      const T a_h = b3 * dv, a_hx = b3 * u, a_hy = b3 * v;
      const T a_q = T(0.5) * (b3 * rt + a_hx * rx + a_hy * ry + a_h * rho);
      yb[0][0] = c0 * dv + b1 * du + b2 * dvv + b3 * (u * ut + v * vt) + a_hx * (u * ux + v * vx) +
                 a_hy * (u * uy + v * vy) + a_h * hq;
      yb[0][1] = c0 * u + a_hx * hq;
      yb[0][2] = c0 * v + a_hy * hq;
      yb[0][3] = c0 + b3 * hq;
      yb[1][0] = c0 * rx + b1 * (r[0] + rho * ux) + b2 * rho * vx + b3 * (rho * ut + hx) + a_hx * rho * ux +
                 a_hy * rho * uy + T(2) * u * a_q;
      yb[1][1] = c0 * rho + b1 * rho * u + b3 * h + a_hx * rho * u;
      yb[1][2] = b1 * rho * v + a_hy * rho * u;
      yb[1][3] = b1 * rho + b3 * rho * u;
      yb[2][0] = c0 * ry + b1 * rho * uy + b2 * (r[0] + rho * vy) + b3 * (rho * vt + hy) + a_hx * rho * vx +
                 a_hy * rho * vy + T(2) * v * a_q;
      yb[2][1] = b2 * rho * u + a_hx * rho * v;
      yb[2][2] = c0 * rho + b2 * rho * v + b3 * h + a_hy * rho * v;
      yb[2][3] = b2 * rho + b3 * rho * v;
      yb[3][0] = a_h * k1;
      yb[3][1] = b1 + a_hx * k1;
      yb[3][2] = b2 + a_hy * k1;
      yb[3][3] = b3 * k;
      break;
    }
    default:
      break;
  }
}

__device__ __forceinline__ void residual_point(const PdeDev& pde, int lapch, const float (&y)[kMaxOut][4],
                                               float (&r)[kMaxOut], float (&yb)[kMaxOut][4]) {
  residual_point_t<float, float>(pde.pde_id, pde.coef, pde.seed_scale, y, r, yb);
  (void)lapch;
}

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Locate the segment of a padded point index.
__device__ __forceinline__ int seg_of(const SegDev& seg, int64_t p) {
  int s = 0;
#pragma unroll 1
  for (int k = 1; k < seg.n_seg; ++k)
    if (p >= seg.start[k]) s = k;
  return s;
}

// Fourier-feature jets of feature j (< m) for point x: cos block and sin block, channels
// 0..3 (Sec. 2.6.1: gamma = [cos(xB), sin(xB)], derivatives by the chain rule).
// B: the Fourier matrix, d_in x n_freq (global memory or a staged copy in LDS)
__device__ __forceinline__ void rff_jets(const NetDev& net, const float* B, const float4 x, int j, f4& cj, f4& sj) {
  const int m = net.n_freq;
  float b0 = B[j], b1 = net.d_in > 1 ? B[m + j] : 0.0f, b2 = net.d_in > 2 ? B[2 * m + j] : 0.0f;
  float v = x.x * b0 + x.y * b1 + x.z * b2;
  float bl = 0.0f;
  if (net.lap_mask & 1) bl += b0 * b0;
  if (net.lap_mask & 2) bl += b1 * b1;
  if (net.lap_mask & 4) bl += b2 * b2;
  float sn, cs;
  sincos_fast(v, sn, cs);
  cj.x = cs;
  sj.x = sn;
  cj.y = -sn * b0;
  sj.y = cs * b0;
  cj.z = net.d_in > 1 ? -sn * b1 : 0.0f;
  sj.z = net.d_in > 1 ? cs * b1 : 0.0f;
  if (net.d_in > 2) {
    cj.w = -sn * b2;
    sj.w = cs * b2;
  } else if (net.lapch == 3) {
    cj.w = -cs * bl;
    sj.w = -sn * bl;
  } else {
    cj.w = 0.0f;
    sj.w = 0.0f;
  }
}

__device__ __forceinline__ void wait_async() { __builtin_amdgcn_s_waitcnt(0); }

// Strict periodic embedding (Sec. 2.6.3): jets of the features of one point, channels
// value, d/dx_k in channel 1 + k, and in channel 3 the Laplacian over lap_mask when the PDE
// has one (two inputs).  Input k of periodic_mask gives the pair cos(omega_k x_k),
// sin(omega_k x_k), whose only derivative is in x_k; every other input passes through.
// The jets sit in fixed slots so that every index is a compile-time constant (no private
// array in scratch memory): slots 2k and 2k + 1 belong to input k (cos and sin, or the input
// itself and an empty slot).  dw (optional): derivative of each slot's jet with respect to
// omega_k (zero for pass-through inputs).
__device__ __forceinline__ void periodic_jets(int d_in, int periodic_mask, int lap_mask, bool lap,
                                              const float* omega, float4 x, f4 (&ej)[6], f4* dw) {
  const float xs[3] = {x.x, x.y, x.z};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ch = 1 + k;
    f4 c = f4{0.f, 0.f, 0.f, 0.f}, sn = f4{0.f, 0.f, 0.f, 0.f};
    f4 dc = f4{0.f, 0.f, 0.f, 0.f}, ds = f4{0.f, 0.f, 0.f, 0.f};
    if (k < d_in) {
      if (!((periodic_mask >> k) & 1)) {
        c[0] = xs[k];
        c[ch] = 1.0f;
      } else {
        const float w = omega[k], xk = xs[k];
        float sv, cv;
        sincos_fast(w * xk, sv, cv);
        const bool inlap = lap && ((lap_mask >> k) & 1);
        c[0] = cv;
        sn[0] = sv;
        c[ch] = -w * sv;
        sn[ch] = w * cv;
        if (inlap) {
          c[3] = -w * w * cv;
          sn[3] = -w * w * sv;
        }
        if (dw) {
          dc[0] = -xk * sv;
          ds[0] = xk * cv;
          dc[ch] = -sv - w * xk * cv;
          ds[ch] = cv - w * xk * sv;
          if (inlap) {
            dc[3] = -2.0f * w * cv + w * w * xk * sv;
            ds[3] = -2.0f * w * sv - w * w * xk * cv;
          }
        }
      }
    }
    ej[2 * k] = c;
    ej[2 * k + 1] = sn;
    if (dw) {
      dw[2 * k] = dc;
      dw[2 * k + 1] = ds;
    }
  }
}

// Feature index (column of the first layer's weights) of a periodic_jets slot, or -1 for an
// empty slot.  Wave-uniform.
__device__ __forceinline__ int periodic_feature(int d_in, int periodic_mask, int slot) {
  const int k = slot >> 1;
  if (k >= d_in) return -1;
  int base = 0;
  for (int j = 0; j < k; ++j) base += (periodic_mask >> j) & 1 ? 2 : 1;
  if (slot & 1) return (periodic_mask >> k) & 1 ? base + 1 : -1;
  return base;
}

// Work-group barrier for LDS traffic: this wave's LDS operations complete (lgkmcnt 0), then
// s_barrier.  Unlike __syncthreads it does not wait for the wave's outstanding vector-memory
// operations (global stores, staged copies), which keep running across the barrier; the
// empty asm statements keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void barrier_lds() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // gfx9 encoding: vmcnt 63, expcnt 7, lgkmcnt 0
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// ================================================================== forward

// Compile-time shape of the forward tile: hidden width bound H, tile points P.
template <int H, int P, int NW = kWaves>
struct FwdShape {
  static constexpr int CPB = P / 4;                    // 16-row cp blocks per tile
  static constexpr int NBMAX = H / 16;                 // neuron blocks
  static constexpr int WN = NBMAX < NW ? NBMAX : NW;
  static constexpr int WC = NW / WN;
  static constexpr int NBW = (NBMAX + WN - 1) / WN;    // neuron blocks per wave
  static constexpr int CBW = CPB / WC;                 // cp blocks per wave
  static_assert(CPB % WC == 0, "tile too small for the wave split");
};

// LDS of the forward tile body.
struct FwdLds {
  char* X;       // layer-input tile (4P rows)
  char* X2;      // second layer-input tile (16-point tiles), else X
  float4* PT;    // tile points
  float* YJ;     // [P][kMaxOut][4] output jets
  float* YB;     // [P][kMaxOut][4] output-jet adjoints
  float* RED;    // [waves][8] wave partial sums (loss terms, then output-bias adjoints)
  double* LOSS;  // [kMaxTerms] sums of squares (FP64, per work item)
  double* WL;    // [WC][kMaxOut][H] output-layer weight-gradient sums
  double* BL;    // [kMaxOut] output-layer bias-gradient sums
  float* BF;     // Fourier matrix, d_in x n_freq (staged once per launch)
  char* OW;      // output-layer weight fragments of the lanes that carry an output:
                 // [chunk < 8][g < 4][output < kMaxOut][32 B] (staged once per launch)
};

template <int H, int P, int NW = kWaves>
__device__ __forceinline__ FwdLds fwd_carve(char* smem, int rs) {
  FwdLds s;
  s.X = smem;
  s.X2 = fwd_double_x(P) ? smem + (size_t)4 * P * rs : smem;
  s.PT = reinterpret_cast<float4*>(smem + (size_t)4 * P * rs * (fwd_double_x(P) ? 2 : 1));
  s.YJ = reinterpret_cast<float*>(s.PT + P);
  s.YB = s.YJ + P * 4 * kMaxOut;
  s.RED = s.YB + P * 4 * kMaxOut;
  s.LOSS = reinterpret_cast<double*>(s.RED + NW * 8);
  s.WL = s.LOSS + kMaxTerms;
  s.BL = s.WL + FwdShape<H, P, NW>::WC * kMaxOut * H;
  s.BF = reinterpret_cast<float*>(s.BL + kMaxOut);
  s.OW = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(s.BF + 3 * kMaxFreq) + 15) & ~(uintptr_t)15);
  return s;
}

// Zero the per-launch sums and stage the Fourier matrix (read by every tile's embedding).
template <int H, int P, int NW = kWaves>
__device__ __forceinline__ void fwd_begin(const FwdLds& s, const NetDev& net) {
  constexpr int NT = 64 * NW;
  for (int i = threadIdx.x; i < kMaxTerms; i += NT) s.LOSS[i] = 0.0;
  for (int i = threadIdx.x; i < FwdShape<H, P, NW>::WC * kMaxOut * H + kMaxOut; i += NT) s.WL[i] = 0.0;
  for (int i = threadIdx.x; i < net.d_in * net.n_freq; i += NT) s.BF[i] = net.B[i];
  // output layer: of each 16-lane group only lanes 0 .. d_out - 1 carry a column
  const LayerDev& lo = net.layer[net.L];
  for (int i = threadIdx.x; i < kOutLds / 4; i += NT) {
    const int w = i & 7, r = i >> 3, o = r % kMaxOut, g = (r / kMaxOut) & 3, kc = r / (4 * kMaxOut);
    uint32_t v = 0;
    if (kc < lo.kci && o < net.d_out)
      v = reinterpret_cast<const uint32_t*>(lo.wf + ((size_t)kc * 64 + 16 * g + o) * 32)[w];
    reinterpret_cast<uint32_t*>(s.OW)[i] = v;
  }
}

// Write the accumulated sums of a run of tiles: loss terms, and (with the gradient) the
// output layer's weight and bias sums in its [d_out][n_L] then [d_out] layout.
template <int H, int P, int NW = kWaves>
__device__ __forceinline__ void fwd_end(const FwdLds& s, double* loss_slot, double* out_slot, int dout, int nL,
                                        bool with_grad) {
  constexpr int NT = 64 * NW;
  __syncthreads();
  for (int i = threadIdx.x; i < kMaxTerms; i += NT) loss_slot[i] = s.LOSS[i];
  if (with_grad) {
    for (int i = threadIdx.x; i < dout * nL; i += NT) {
      const int o = i / nL, n = i - o * nL;
      double t = 0.0;
      for (int c = 0; c < FwdShape<H, P, NW>::WC; ++c) t += s.WL[(c * kMaxOut + o) * H + n];
      out_slot[i] = t;
    }
    for (int o = threadIdx.x; o < dout; o += NT) out_slot[dout * nL + o] = s.BL[o];
  }
}

// What a tile is: residual points (kind 0) or one value-supervision set (kind 1).
struct TileSeg {
  int kind;
  int nvalid;            // valid points of the tile (the rest is padding)
  int term;              // first loss term this tile adds to
  const float* targets;  // kind 1: targets of the tile's first point (d_out per point)
  int out_mask;
  float lam;             // kind 1: 2 lambda / N_s
  float* residual;       // kind 0: residual of the tile's first point, or null
};

// One tile of P points through the whole forward pass: embedding jets, hidden layers
// (stash of every pre-activation), output layer, residual, loss partial sums, output-jet
// seed and (with the gradient) the output layer's backward.  pts: the tile's points;
// zs: stash of hidden layer 0 with zs_stride floats between layers; zb0: adjoint of the
// last hidden layer; cb_st: first cp block of this tile in those buffers; amx: running
// largest magnitude of the adjoint written to zb0 (FP16X3 only).
template <int PREC, int ACT, int H, int P, int NW = kWaves>
__device__ __forceinline__ void fwd_tile(const NetDev& net, const PdeDev& pde, const float4* pts, float* zs,
                                         int64_t zs_stride, float* zb0, int64_t cb_st, const TileSeg& sg, int ld,
                                         bool with_grad, const FwdLds& s, float& amx) {
  using S = FwdShape<H, P, NW>;
  constexpr int NT = 64 * NW;
  static_assert(P <= NT, "one thread per tile point");
  using Pr = Prec<PREC>;
  constexpr int CPB = S::CPB, NBW = S::NBW, CBW = S::CBW, WN = S::WN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int wn = wave % WN, wc = wave / WN;
  const int L = net.L, dout = net.d_out;
  char* X = s.X;
  float lw1, lw2;
  lap_weights(net, lw1, lw2);
  const LayerDev& lout = net.layer[L];

  barrier_lds();  // the previous user of the LDS is done
  for (int p = tid; p < P; p += NT) s.PT[p] = pts[p];
  barrier_lds();

  f4 acc[NBW][CBW];
  // ---- layer 0
  const LayerDev& l0 = net.layer[0];
  if (net.n_freq == 0 && !net.periodic_mask) {
    // identity embedding: z = W x + b on the value channel, d z / d x_k = W[:, k]
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      const int nb = wn + WN * i;
      const bool ok = nb * 16 < l0.n_out;
      const int n = ok ? 16 * nb + l16 : 0;
      float w[3] = {0.f, 0.f, 0.f};
      float bn = 0.f;
      if (ok) {
        for (int k = 0; k < net.d_in; ++k) w[k] = l0.w[n * net.d_in + k];
        bn = l0.b[n];
      }
#pragma unroll
      for (int c = 0; c < CBW; ++c) {
        const float4 x = s.PT[4 * (wc * CBW + c) + g];
        f4 z;
        z.x = bn + w[0] * x.x + w[1] * x.y + w[2] * x.z;
        z.y = w[0];
        z.z = w[1];
        z.w = net.d_in > 2 ? w[2] : 0.0f;
        acc[i][c] = z;
      }
    }
  } else {
    if (net.periodic_mask) {
      // periodic embedding (Sec. 2.6.3): the e <= 6 feature jets of each point into the
      // tile, the rest of the first 32-wide reduction chunk cleared (its weights are zero,
      // but the tile holds the previous layer's jets), then z = W e + b as for Fourier
      // features; lane (g, l16) takes point 4 pb + g and column l16 or 16 + l16
      for (int pb = wave; pb < P / 4; pb += NW) {
        const int p = 4 * pb + g;
        f4 ej[6];
        periodic_jets(net.d_in, net.periodic_mask, net.lap_mask, net.lapch >= 0, net.omega, s.PT[p], ej, nullptr);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int col = 16 * h + l16;
          f4 v = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < 6; ++q)
            if (periodic_feature(net.d_in, net.periodic_mask, q) == col) v = ej[q];
          Tile<PREC>::put(X, ld, p, col, v);
        }
      }
    } else {
      // Fourier-feature jets into the tile, then z = W gamma + b
      // blocks of 4 points x 16 frequencies per wave: lane (g, l16) takes point 4 pb + g,
      // frequency 16 jb + l16, the write pattern of an accumulator block
      const int m = net.n_freq;
      const int nj = m >> 4;
      for (int b = wave; b < (P / 4) * nj; b += NW) {
        const int pb = b / nj, jb = b - (b / nj) * nj;
        const int p = 4 * pb + g, j = 16 * jb + l16;
        f4 cj, sj;
        rff_jets(net, s.BF, s.PT[p], j, cj, sj);
        Tile<PREC>::put(X, ld, p, j, cj);
        Tile<PREC>::put(X, ld, p, m + j, sj);
      }
    }
    barrier_lds();
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int c = 0; c < CBW; ++c) acc[i][c] = f4{0.f, 0.f, 0.f, 0.f};
    {
      int blk[NBW];
#pragma unroll
      for (int i = 0; i < NBW; ++i) blk[i] = min(wn + WN * i, l0.nbo - 1);
      gemm_tile<PREC, NBW, CBW, 8, true>(acc, X, ld, wc * CBW, l0.wf, l0.kci, blk, lane);
    }
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      const int nb = wn + WN * i;
      const float bn = nb < l0.nbo ? l0.b[16 * nb + l16] : 0.0f;
#pragma unroll
      for (int c = 0; c < CBW; ++c) acc[i][c].x += bn;
    }
  }

  // Small tiles keep the last hidden layer's pre-activation jets in the accumulators until
  // the output layer's backward below; no later kernel reads that layer's stash, so it is
  // written only when the jets are read back from it here.
  constexpr bool kLive = CBW <= 8;
  // Early weight loads (the next layer's first chunks before the stash stores, the output
  // layer's chunks all at once) cost registers; the bf16x3 shapes with at most 8 cp blocks
  // per wave have them to spare.
  constexpr bool kPre = is_split(PREC) && CBW <= 8 && NBW <= 2;

  // ---- hidden layers: acc holds z of layer j
  for (int j = 0; j < L; ++j) {
    const LayerDev& lj = net.layer[j];
    const int nbs = lj.n_out / 16;
    // the next layer's first weight chunks and biases load before this layer's stash stores,
    // so that the next product's first waits leave those stores in flight
    Raw pre0[NBW], pre1[NBW];
    int nblk[NBW];
    float nbias[NBW];
    const bool next = j + 1 < L;
    if (next) {
      const LayerDev& ln = net.layer[j + 1];
#pragma unroll
      for (int i = 0; i < NBW; ++i) {
        const int nb = wn + WN * i;
        nblk[i] = min(nb, ln.nbo - 1);
        nbias[i] = nb < ln.nbo ? ln.b[16 * nb + l16] : 0.0f;
      }
      if (kPre) load_first_chunks<NBW>(pre0, pre1, ln.wf, ln.kci, nblk, lane);
    }
    // layer j's activations go to XA; with one tile (XA == X) every wave must first be done
    // reading the layer input from it, with two they go to the tile the product did not read
    char* XA = (j & 1) ? X : s.X2;
    if (!fwd_double_x(P)) barrier_lds();
    // activation jets into XA, each fragment's stash store issued beside its activation (the
    // stores overlap the vector-ALU work instead of forming a burst of their own); the stores
    // are issued unconditionally and switched off by offset (FragStore)
    {
      const bool keep = with_grad && !(kLive && j == L - 1);
      const FragStore st(zs + j * zs_stride, cb_st, CPB, nbs);
#pragma unroll
      for (int i = 0; i < NBW; ++i) {
        const int nb = wn + WN * i;
        const int n = 16 * nb + l16;
#pragma unroll
        for (int c = 0; c < CBW; ++c) {
          const int cb = wc * CBW + c;
          st.put(cb, nb, lane, acc[i][c], keep && nb < nbs);
          if (nb < nbs) {
            float s0, s1, s2, s3;
            act_eval<ACT>(acc[i][c].x, net.w0, s0, s1, s2, s3);
            const f4 a = jet_act<(ACT & kLapFlag) != 0>(acc[i][c], s0, s1, s2, lw1, lw2);
            Tile<PREC>::put(XA, ld, 4 * cb + g, n, a);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    barrier_lds();
    if (next) {
      const LayerDev& ln = net.layer[j + 1];
#pragma unroll
      for (int i = 0; i < NBW; ++i)
#pragma unroll
        for (int c = 0; c < CBW; ++c) acc[i][c] = f4{0.f, 0.f, 0.f, 0.f};
      gemm_tile<PREC, NBW, CBW, 8, true, kPre>(acc, XA, ld, wc * CBW, ln.wf, ln.kci, nblk, lane, pre0, pre1);
#pragma unroll
      for (int i = 0; i < NBW; ++i)
#pragma unroll
        for (int c = 0; c < CBW; ++c) acc[i][c].x += nbias[i];
    }
  }

  // ---- output layer (d_out <= kMaxOut columns of one 16-wide block): waves over cp blocks, the
  // weight fragments from their staged copy in LDS (zero on the lanes without an output)
  const char* XL = ((L - 1) & 1) ? X : s.X2;  // the last hidden layer's activations
  const float obias = l16 < dout ? lout.b[l16] : 0.0f;
  for (int cb = wave; cb < CPB; cb += NW) {
    f4 y = f4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < lout.kci; ++kc) {
      const Raw a = Tile<PREC>::load(XL, ld, cb, kc, lane);
      Raw bw;
      bw.a = make_uint4(0, 0, 0, 0);
      bw.b = bw.a;
      if (l16 < kMaxOut) bw = *reinterpret_cast<const Raw*>(s.OW + ((kc * 4 + g) * kMaxOut + l16) * 32);
      Pr::mma(y, a, bw);
    }
    if (l16 < dout) {
      y.x += obias;
      float* dst = s.YJ + ((4 * cb + g) * kMaxOut + l16) * 4;
      *reinterpret_cast<float4*>(dst) = to_float4(y);
    }
  }
  barrier_lds();

  // ---- residual (or supervision misfit), loss partial sums and the output-jet seed
  float part[kMaxOut] = {};
  float ybv[kMaxOut] = {};  // value-channel output adjoints: the output bias gradient
  if (tid < P) {
    const int p = tid;
    float y[kMaxOut][4], yb[kMaxOut][4];
#pragma unroll
    for (int o = 0; o < kMaxOut; ++o)
#pragma unroll
      for (int c = 0; c < 4; ++c) y[o][c] = o < dout ? s.YJ[(p * kMaxOut + o) * 4 + c] : 0.0f;
    const bool valid = p < sg.nvalid;
    if (sg.kind == 0) {
      float r[kMaxOut];
      residual_point(pde, net.lapch, y, r, yb);
      if (valid) {
        for (int c = 0; c < pde.n_res; ++c) part[c] = r[c] * r[c];
        if (sg.residual)
          for (int c = 0; c < pde.n_res; ++c) sg.residual[(int64_t)p * pde.n_res + c] = r[c];
      }
    } else {
#pragma unroll
      for (int o = 0; o < kMaxOut; ++o)
#pragma unroll
        for (int c = 0; c < 4; ++c) yb[o][c] = 0.0f;
      if (valid) {
        for (int o = 0; o < dout; ++o) {
          if (!(sg.out_mask & (1 << o))) continue;
          const float d = y[o][0] - sg.targets[(int64_t)p * dout + o];
          part[0] += d * d;
          yb[o][0] = sg.lam * d;
        }
      }
    }
    if (!valid) {
#pragma unroll
      for (int o = 0; o < kMaxOut; ++o)
#pragma unroll
        for (int c = 0; c < 4; ++c) yb[o][c] = 0.0f;
    }
#pragma unroll
    for (int o = 0; o < kMaxOut; ++o) {
      *reinterpret_cast<float4*>(s.YB + (p * kMaxOut + o) * 4) = make_float4(yb[o][0], yb[o][1], yb[o][2], yb[o][3]);
      ybv[o] = yb[o][0];
    }
  }
  static_assert(kMaxOut <= 4, "RED holds 4 loss terms and 4 output-bias sums per wave");
#pragma unroll
  for (int k = 0; k < kMaxOut; ++k) {
    const float v = wave_sum(part[k]);
    const float u = wave_sum(ybv[k]);
    if (lane == 0) {
      s.RED[wave * 8 + k] = v;
      s.RED[wave * 8 + 4 + k] = u;
    }
  }
  barrier_lds();
  {
    // one thread per loss term and per output bias, each summing the waves in order
    const int nterm = sg.kind == 0 ? pde.n_res : 1;
    if (tid < nterm) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += (double)s.RED[w * 8 + tid];
      s.LOSS[sg.term + tid] += t;
    } else if (with_grad && tid >= 4 && tid < 4 + dout) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += (double)s.RED[w * 8 + tid];
      s.BL[tid - 4] += t;
    }
  }

  // ---- output layer backward: W_out / b_out sums, adjoint of the last hidden layer
  if (with_grad) {
    const int nL = lout.n_in;
    const int nbs = nL / 16;
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      const int nb = wn + WN * i;
      if (nb >= nbs) continue;
      const int n = 16 * nb + l16;
      float wo[kMaxOut], wsum[kMaxOut] = {};
#pragma unroll
      for (int o = 0; o < kMaxOut; ++o) wo[o] = o < dout ? lout.w[o * nL + n] : 0.0f;
      // pre-activation jets of the last hidden layer: still in the accumulators when the
      // tile is small, else read back from the stash (fewer live registers)
#pragma unroll(kLive ? CBW : 1)
      for (int c = 0; c < CBW; ++c) {
        const int cb = wc * CBW + c;
        const int p = 4 * cb + g;
        const f4 z = kLive ? acc[i][c] : to_f4(*jet_frag(zs + (L - 1) * zs_stride, cb_st + cb, nb, nbs, lane));
        float s0, s1, s2, s3;
        act_eval<ACT>(z.x, net.w0, s0, s1, s2, s3);
        const f4 a = jet_act<(ACT & kLapFlag) != 0>(z, s0, s1, s2, lw1, lw2);
        f4 ab = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int o = 0; o < kMaxOut; ++o) {
          if (o >= 3 && o >= dout) continue;  // a fourth output only where there is one
          const f4 yb = to_f4(*reinterpret_cast<const float4*>(s.YB + (p * kMaxOut + o) * 4));
          ab += yb * wo[o];
          wsum[o] += yb.x * a.x + yb.y * a.y + yb.z * a.z + yb.w * a.w;
        }
        const f4 zb = jet_act_adj<(ACT & kLapFlag) != 0>(z, ab, s1, s2, s3, lw1, lw2);
        __builtin_nontemporal_store(zb, reinterpret_cast<f4*>(jet_frag(zb0, cb_st + cb, nb, nbs, lane)));
        if constexpr (PREC == kFP16X3) amx = fmaxf(amx, jet_absmax(zb));
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int o = 0; o < kMaxOut; ++o) {
        float v = wsum[o];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == 0 && o < dout) s.WL[(wc * kMaxOut + o) * H + n] += (double)v;
      }
    }
  }
}

// ================================================================== backward (one layer)

template <int NOB, int NIB, int PB>
struct BwdShape {
  static constexpr int CPB = PB / 4;
  // weight-gradient split: WO waves over output blocks x WI over input blocks
  static constexpr int WO = NOB < kWaves ? NOB : kWaves;
  static constexpr int WI = kWaves / WO;
  static constexpr int NOBW = (NOB + WO - 1) / WO;
  static constexpr int NIBW = (NIB + WI - 1) / WI;
  // input-adjoint split: WA waves over input blocks x WCA over cp blocks
  static constexpr int WA = NIB < kWaves ? NIB : kWaves;
  static constexpr int WCA = kWaves / WA;
  static constexpr int NIBA = (NIB + WA - 1) / WA;
  static constexpr int CBA = CPB / WCA;
  static_assert(CPB % 2 == 0 && CPB % WCA == 0, "sub-tile too small");
};

// LDS regions of the layer backward for sub-tiles of PB points:
//   ZB  staged adjoint fragments of the layer output (PB x n_out jets, fragment-major),
//   ZP  staged pre-activation fragments of the layer input (PB x n_in), hidden layers only,
//   Q   layer-input jets in the Q layout (B operand of the weight gradient),
//   R   output adjoint in the R layout (A operand of the input adjoint), hidden layers only.
struct BwdLds {
  char *ZB, *ZP, *Q, *R;
};

__host__ __device__ constexpr size_t bwd_lds_bytes(int PB, int n_in, int n_out, bool with_prev) {
  return (size_t)PB * n_out * 16 + (with_prev ? (size_t)PB * n_in * 16 : 0) + (size_t)n_in * q_stride(4 * PB) +
         (with_prev ? (size_t)4 * PB * r_stride(n_out) : 0);
}

__device__ __forceinline__ BwdLds bwd_carve(char* smem, int PB, int n_in, int n_out, bool with_prev) {
  BwdLds s;
  s.ZB = smem;
  s.ZP = s.ZB + (size_t)PB * n_out * 16;
  s.Q = s.ZP + (with_prev ? (size_t)PB * n_in * 16 : 0);
  s.R = s.Q + (size_t)n_in * q_stride(4 * PB);
  return s;
}

// Start an asynchronous copy of `bytes` (a multiple of 1 KiB) contiguous bytes of device
// memory into LDS: every wave moves 1 KiB per instruction, 16 bytes per lane landing at
// consecutive LDS addresses.  Completion: s_waitcnt vmcnt(0), then a barrier.
__device__ __forceinline__ void async_copy(char* dst, const char* src, int bytes) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int off = wave * 1024; off < bytes; off += kWaves * 1024)
    __builtin_amdgcn_global_load_lds(src + off + lane * 16,
                                     (__attribute__((address_space(3))) void*)(dst + off), 16, 0, 0);
}


// Linear layer `layer`'s backward over `count` sub-tiles of PB points, sub-tile k being
// number s0 + k * stride: weight-gradient sums (accw, bsum, kept by the caller), and for
// layers with a predecessor the input adjoint and the activation adjoint (zb_out).  The
// jets of sub-tile k + 1 are copied into LDS while sub-tile k is computed.  pts: points of
// sub-tile 0 of the index space (Fourier embedding only).  asc: scale of the output adjoint
// in its 16-bit operands (adj_scale; the weight-gradient sums come out scaled by it, the
// input adjoint is scaled back); amx: running largest magnitude of what goes to zb_out.
template <int PREC, int ACT, int NOB, int NIB, int PB>
__device__ __forceinline__ void bwd_range(const NetDev& net, int layer, const float4* pts, int64_t s0, int64_t stride,
                                          int64_t count, const float* zb_in, float* zb_out, const float* z_prev,
                                          char* smem,
                                          f4 (&accw)[BwdShape<NOB, NIB, PB>::NOBW][BwdShape<NOB, NIB, PB>::NIBW],
                                          float (&bsum)[BwdShape<NOB, NIB, PB>::NOBW], float asc, float& amx,
                                          double* g0_slot = nullptr) {
  using S = BwdShape<NOB, NIB, PB>;
  using Pr = Prec<PREC>;
  constexpr int CPB = S::CPB, NOBW = S::NOBW, NIBW = S::NIBW, NIBA = S::NIBA, CBA = S::CBA;
  // g0_slot (layer 1 over an identity embedding): the first layer's weight and bias sums
  // are formed here from the input adjoint, which is then not written (slot layout
  // [n_in][d_in] then [n_in]).  Each lane adds its terms in FP64: a work-group's range
  // holds thousands of points per lane and neuron.
  double g0s[NIBA][4];
#pragma unroll
  for (int q = 0; q < NIBA; ++q) g0s[q][0] = g0s[q][1] = g0s[q][2] = g0s[q][3] = 0.0;
  constexpr int WO = S::WO, WA = S::WA;
  const LayerDev& ly = net.layer[layer];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int n_in = ly.n_in, n_out = ly.n_out;
  const int nob = n_out / 16, nib = n_in / 16;
  const bool has_prev = z_prev != nullptr;
  const int rld = Tile<PREC>::ld(n_out, PB);
  float lw1, lw2;
  lap_weights(net, lw1, lw2);
  const int qs = q_stride(4 * PB);
  const BwdLds L = bwd_carve(smem, PB, n_in, n_out, has_prev);
  const int wo = wave % WO, wi = wave / WO;
  const int wa = wave % WA, wca = wave / WA;
  const int zb_bytes = CPB * nob * 1024, zp_bytes = CPB * nib * 1024;
  auto zb_src = [&](int64_t s) { return reinterpret_cast<const char*>(zb_in) + s * zb_bytes; };
  auto zp_src = [&](int64_t s) { return reinterpret_cast<const char*>(z_prev) + s * zp_bytes; };
  auto frag = [&](const char* base, int cb, int nb, int nbs) {
    return to_f4(*reinterpret_cast<const float4*>(base + ((size_t)(cb * nbs + nb) * 64 + lane) * 16));
  };

  if (count <= 0) {
    if (g0_slot)
      for (int i = tid; i < n_in * (net.d_in + 1); i += kThreads) g0_slot[i] = 0.0;
    return;
  }
  // input-adjoint weight fragments: at widths up to 128 (at most 4 per lane) loaded once
  // for the whole range and kept in registers, wider layers stream them per sub-tile
  constexpr int KCM = NOB / 2 > 0 ? NOB / 2 : 1;
  constexpr bool kResW = NIBA * KCM <= 4;
  Raw wres[NIBA][kResW ? KCM : 1];
  if constexpr (kResW) {
    if (has_prev) {
#pragma unroll
      for (int q = 0; q < NIBA; ++q)
#pragma unroll
        for (int kc = 0; kc < KCM; ++kc)
          if (kc < ly.kco) wres[q][kc] = glob_frag(ly.wb, min(wa + WA * q, nib - 1), kc, ly.kco, lane);
    }
  }
  __syncthreads();  // the previous user of the LDS is done
  async_copy(L.ZB, zb_src(s0), zb_bytes);
  if (has_prev) async_copy(L.ZP, zp_src(s0), zp_bytes);

  for (int64_t k = 0; k < count; ++k) {
    const int64_t s = s0 + k * stride;
    wait_async();
    barrier_lds();  // sub-tile s is in ZB / ZP; the previous sub-tile is done with R and Q
    // (1) output adjoint: R layout for the input adjoint, A operands of the weight gradient
    if (has_prev) {
      for (int f = wave; f < CPB * nob; f += kWaves) {
        const int cb = f % CPB, ob = f / CPB;
        const f4 zb = frag(L.ZB, cb, ob, nob);
        const int o = 16 * ob + l16;
        Tile<PREC>::put(L.R, rld, 4 * cb + g, o, ascale<PREC>(zb, asc));
      }
    }
    Raw ao[CPB / 2][NOBW];
#pragma unroll
    for (int cc = 0; cc < CPB / 2; ++cc)
#pragma unroll
      for (int i = 0; i < NOBW; ++i) {
        const int ob = min(wo + WO * i, nob - 1);  // clamped duplicates are never stored
        const f4 v0 = frag(L.ZB, 2 * cc, ob, nob), v1 = frag(L.ZB, 2 * cc + 1, ob, nob);
        bsum[i] += v0.x + v1.x;
        const f4 w0 = ascale<PREC>(v0, asc), w1 = ascale<PREC>(v1, asc);
        const float f[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        ao[cc][i] = Pr::make(f);
      }
    barrier_lds();  // R complete; ZB no longer read
    if (k + 1 < count) async_copy(L.ZB, zb_src(s + stride), zb_bytes);
    const int64_t cb0 = s * CPB;
    if (has_prev) {
      // (2) adjoint of the layer input: abar[cp][i] = sum_o zbar[cp][o] W[o][i]
      f4 acca[NIBA][CBA];
#pragma unroll
      for (int q = 0; q < NIBA; ++q)
#pragma unroll
        for (int c = 0; c < CBA; ++c) acca[q][c] = f4{0.f, 0.f, 0.f, 0.f};
      if constexpr (kResW) {
#pragma unroll
        for (int kc = 0; kc < KCM; ++kc) {
          if (kc >= ly.kco) break;
          Raw a[CBA], b[NIBA];
#pragma unroll
          for (int c = 0; c < CBA; ++c) a[c] = Tile<PREC>::load(L.R, rld, wca * CBA + c, kc, lane);
#pragma unroll
          for (int q = 0; q < NIBA; ++q) b[q] = wres[q][kc];
          Pr::template mma_tile<NIBA, CBA>(acca, a, b);
        }
      } else {
        int blk[NIBA];
#pragma unroll
        for (int q = 0; q < NIBA; ++q) blk[q] = min(wa + WA * q, nib - 1);
        gemm_tile<PREC, NIBA, CBA, 8, true>(acca, L.R, rld, wca * CBA, ly.wb, ly.kco, blk, lane);
      }
      // (3) one pass over the layer input's pre-activations: recomputed activation jets
      // into Q (operand of the weight gradient) and the activation adjoint
#pragma unroll
      for (int q = 0; q < NIBA; ++q) {
        const int ib = wa + WA * q;
        if (ib >= nib) continue;
        const int n = 16 * ib + l16;
#pragma unroll
        for (int c = 0; c < CBA; ++c) {
          const int cb = wca * CBA + c;
          const f4 z = frag(L.ZP, cb, ib, nib);
          float s0v, s1v, s2v, s3v;
          act_eval<ACT>(z.x, net.w0, s0v, s1v, s2v, s3v);
          const f4 a = jet_act<(ACT & kLapFlag) != 0>(z, s0v, s1v, s2v, lw1, lw2);
          int unit, pos0;
          q_pos(cb, g, unit, pos0);
          Pr::put4(L.Q + (size_t)n * qs + unit * 32, pos0, a);
          const f4 zb = jet_act_adj<(ACT & kLapFlag) != 0>(z, ascale<PREC>(acca[q][c], 1.0f / asc), s1v, s2v, s3v,
                                                          lw1, lw2);
          if (g0_slot) {
            // the identity input's jets are (x_k, e_k, 0)
            const float4 x = pts[(cb0 + cb) * 4 + g];
            g0s[q][0] += (double)(zb.x * x.x + zb.y);
            g0s[q][1] += (double)(zb.x * x.y + zb.z);
            g0s[q][2] += (double)(zb.x * x.z + zb.w);
            g0s[q][3] += (double)zb.x;
          } else {
            *jet_frag(zb_out, cb0 + cb, ib, nib, lane) = to_float4(zb);
          }
          if constexpr (PREC == kFP16X3) amx = fmaxf(amx, jet_absmax(zb));
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
      // Fourier-feature embedding of the sub-tile's points into Q
      const int m = net.n_freq;
      const float4* sp = pts + s * PB;
      for (int idx = tid; idx < PB * m; idx += kThreads) {
        const int p = idx / m, j = idx - (idx / m) * m;
        f4 cj, sj;
        rff_jets(net, net.B, sp[p], j, cj, sj);
        const int cb = p >> 2, gg = p & 3;
        int unit, pos0;
        q_pos(cb, gg, unit, pos0);
        Pr::put4(L.Q + (size_t)j * qs + unit * 32, pos0, cj);
        Pr::put4(L.Q + (size_t)(m + j) * qs + unit * 32, pos0, sj);
      }
    }
    barrier_lds();  // Q complete; ZP no longer read
    if (has_prev && k + 1 < count) async_copy(L.ZP, zp_src(s + stride), zp_bytes);
    // (4) weight gradient: W_bar[o][i] += sum_cp zbar[cp][o] a[cp][i]
#pragma unroll
    for (int cc = 0; cc < CPB / 2; ++cc)
#pragma unroll
      for (int q = 0; q < NIBW; ++q) {
        const Raw bq = lds_unit(L.Q, 16 * min(wi + S::WI * q, nib - 1) + l16, 4 * cc + g, qs);
#pragma unroll
        for (int i = 0; i < NOBW; ++i) Pr::mma(accw[i][q], ao[cc][i], bq);
      }
  }
  if (g0_slot) {
    // over the lanes of a neuron, then over the waves that share it (fixed order)
    double* red = reinterpret_cast<double*>(smem);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NIBA; ++q) {
      const int ib = wa + WA * q;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double v = g0s[q][k];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == 0 && ib < nib) red[((size_t)wca * n_in + 16 * ib + l16) * 4 + k] = v;
      }
    }
    __syncthreads();
    const int d = net.d_in;
    for (int i = tid; i < n_in; i += kThreads) {
      double t[4] = {0.0, 0.0, 0.0, 0.0};
      for (int w = 0; w < kWaves / WA; ++w)
        for (int k = 0; k < 4; ++k) t[k] += red[((size_t)w * n_in + i) * 4 + k];
      for (int k = 0; k < d; ++k) g0_slot[(size_t)i * d + k] = t[k];
      g0_slot[(size_t)n_in * d + i] = t[3];
    }
  }
}

// Store the weight-gradient sums (FP32 over the run of sub-tiles) as FP64 into a slot laid
// out [n_out][n_in] then [n_out] (bias); the weight sums are multiplied by inv (the
// reciprocal of the adjoint scale, a power of two).
template <int NOB, int NIB, int PB>
__device__ __forceinline__ void bwd_flush(const f4 (&accw)[BwdShape<NOB, NIB, PB>::NOBW][BwdShape<NOB, NIB, PB>::NIBW],
                                          const float (&bsum)[BwdShape<NOB, NIB, PB>::NOBW], double* slot, int n_out,
                                          int n_in, float inv = 1.0f) {
  using S = BwdShape<NOB, NIB, PB>;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int wo = wave % S::WO, wi = wave / S::WO;
  const int nob = n_out / 16, nib = n_in / 16;
#pragma unroll
  for (int i = 0; i < S::NOBW; ++i) {
    const int ob = wo + S::WO * i;
    if (ob >= nob) continue;
#pragma unroll
    for (int k = 0; k < S::NIBW; ++k) {
      const int ib = wi + S::WI * k;
      if (ib >= nib) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        slot[(size_t)(16 * ob + 4 * g + r) * n_in + 16 * ib + l16] = (double)accw[i][k][r] * (double)inv;
    }
    if (wi == 0) {
      float v = bsum[i];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (g == 0) slot[(size_t)n_out * n_in + 16 * ob + l16] = (double)v;
    }
  }
}

// ================================================================== first layer, identity

// W_bar[o][k] = sum_points (zbar0[o] x_k + zbar_{1+k}[o]), b_bar[o] = sum zbar0[o]: the
// identity embedding's jets are (x, unit vectors, 0).  Sums over cp blocks [cb_lo, cb_hi)
// of the adjoint buffer (points pts[4 cb + ...]) into slot [n_out][d_in] then [n_out].
// red: LDS scratch of kWaves * 256 * 4 floats.
__device__ __forceinline__ void grad0_range(const float* zb, const float4* pts, int n_out, int d_in, int64_t cb_lo,
                                            int64_t cb_hi, double* slot, float* red) {
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nob = n_out / 16;
  __syncthreads();
  // every cp block once, all neuron blocks of it together (up to 16 independent loads in
  // flight per wave); per neuron block the sums run over the cp blocks in order
  constexpr int kMaxOb = 16;  // n_out <= 256
  float s[kMaxOb][4];
#pragma unroll
  for (int ob = 0; ob < kMaxOb; ++ob)
#pragma unroll
    for (int k = 0; k < 4; ++k) s[ob][k] = 0.f;
  for (int64_t cb = cb_lo + wave; cb < cb_hi; cb += kWaves) {
    const float4 x = pts[4 * cb + g];
#pragma unroll
    for (int ob = 0; ob < kMaxOb; ++ob) {
      if (ob < nob) {
        const float4 z = *jet_frag(const_cast<float*>(zb), cb, ob, nob, lane);
        s[ob][0] += z.x * x.x + z.y;
        s[ob][1] += z.x * x.y + z.z;
        s[ob][2] += z.x * x.z + z.w;
        s[ob][3] += z.x;
      }
    }
  }
#pragma unroll
  for (int ob = 0; ob < kMaxOb; ++ob) {
    if (ob >= nob) continue;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float v = s[ob][k];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (g == 0) red[(wave * 256 + 16 * ob + l16) * 4 + k] = v;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_out; i += kThreads) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < kWaves; ++w)
      for (int k = 0; k < 4; ++k) t[k] += (double)red[(w * 256 + i) * 4 + k];
    for (int k = 0; k < d_in; ++k) slot[(size_t)i * d_in + k] = t[k];
    slot[(size_t)n_out * d_in + i] = t[3];
  }
}

// First-layer weight gradient with the periodic embedding (Sec. 2.6.3): for every output o
// W_bar[o][j] = sum_points sum_c zbar[o][c] e_j[c], b_bar[o] = sum zbar[o][0], and for the
// features j of trained periods G[o][j] = sum zbar[o][c] d e_j[c] / d omega (the period
// gradient follows from G and W in the reduction).  Four output blocks at a time; per
// block the sums run over the cp blocks in order.  Slot: [n_out][e], [n_out], [n_out][ng].
// red: LDS scratch of kWaves * 64 * 13 floats.
__device__ __forceinline__ void grad0p_range(const Grad0Args& A, int64_t cb_lo, int64_t cb_hi, double* slot,
                                             float* red) {
  const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nob = A.n_out / 16, e = A.e;
  const bool lap = A.lap_mask != 0;
  // slots of trained periods (bits 2k and 2k + 1 for a trained input k)
  int tmask = 0, ng = 0;
  for (int k = 0; k < A.d_in; ++k)
    if ((A.period_train_mask >> k) & 1) {
      tmask |= 3 << (2 * k);
      ng += 2;
    }
  // sums per output, by slot of periodic_jets: sum[q] weights, sum[6] bias, sum[7 + q] the
  // period terms of trained slots
  constexpr int kG = 4;  // output blocks per pass
  for (int og = 0; og < nob; og += kG) {
    float sum[kG][13];
#pragma unroll
    for (int q = 0; q < kG; ++q)
#pragma unroll
      for (int a = 0; a < 13; ++a) sum[q][a] = 0.f;
    for (int64_t cb = cb_lo + wave; cb < cb_hi; cb += kWaves) {
      f4 ej[6], dw[6];
      periodic_jets(A.d_in, A.periodic_mask, A.lap_mask, lap, A.omega, A.pts[4 * cb + g], ej, dw);
#pragma unroll
      for (int q = 0; q < kG; ++q) {
        const int ob = og + q;
        if (ob >= nob) continue;
        const f4 z = to_f4(*jet_frag(const_cast<float*>(A.zb), cb, ob, nob, lane));
#pragma unroll
        for (int j = 0; j < 6; ++j) sum[q][j] += z.x * ej[j].x + z.y * ej[j].y + z.z * ej[j].z + z.w * ej[j].w;
        sum[q][6] += z.x;
#pragma unroll
        for (int f = 0; f < 6; ++f)
          if ((tmask >> f) & 1) sum[q][7 + f] += z.x * dw[f].x + z.y * dw[f].y + z.z * dw[f].z + z.w * dw[f].w;
      }
    }
    __syncthreads();  // red free
#pragma unroll
    for (int q = 0; q < kG; ++q)
#pragma unroll
      for (int a = 0; a < 13; ++a) {
        float v = sum[q][a];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == 0) red[((wave * kG + q) * 16 + l16) * 13 + a] = v;
      }
    __syncthreads();
    for (int i = threadIdx.x; i < kG * 16; i += kThreads) {
      const int o = 16 * og + i;
      if (o >= A.n_out) continue;
      double t[13];
      for (int a = 0; a < 13; ++a) t[a] = 0.0;
      for (int w = 0; w < kWaves; ++w)
        for (int a = 0; a < 13; ++a) t[a] += (double)red[(w * kG * 16 + i) * 13 + a];
      for (int q = 0, j = 0; q < 6; ++q) {
        const int f = periodic_feature(A.d_in, A.periodic_mask, q);
        if (f >= 0) slot[(size_t)o * e + f] = t[q];
        if ((tmask >> q) & 1) slot[(size_t)A.n_out * (e + 1) + (size_t)o * ng + j++] = t[7 + q];
      }
      slot[(size_t)A.n_out * e + o] = t[6];
    }
  }
}

// Launch helpers.
// Dynamic LDS above 64 KiB has to be allowed per kernel.
template <typename K>
inline int set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return 0;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes) == hipSuccess ? 0 : -5;
}
inline int launch_status(hipError_t e) { return e == hipSuccess ? 0 : -5; }

// ================================================================== split-role pieces
// Shapes and matrix-core loops of the hidden-layer backward whose input-adjoint work keeps
// the layer's weights resident in registers and whose weight-gradient work keeps the sums
// resident (the two roles of k_backward_split, and the two passes of the batched launch).
template <int NOB, int NIB, int PB>
struct SplitShape {
  static constexpr int CPB = PB / 4;
  static constexpr int NIBW = NIB / 8;   // input blocks per wave
  static constexpr int NOBC = (NOB + 7) / 8;  // output blocks converted per wave
  static constexpr int KC = NOB / 2;     // reduction chunks of the input adjoint (n_out / 32)
  static constexpr int NSTORE = NIBW * CPB;  // adjoint stores per lane and sub-tile
  static_assert(NIB % 8 == 0 && CPB % 2 == 0, "split backward shape");
};

// s_waitcnt with only the vector-memory count bounded (gfx9 encoding: vmcnt in bits 3:0
// and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Input-adjoint product of the split backward's first role, with the copy of the next
// sub-tile's adjoint into STG started first.  STG and R are distinct LDS regions; the
// restrict qualifiers let the compiler's wait insertion see that the tile reads do not
// depend on the copy.
template <int PREC, int NIBW, int CPB, int KC>
__device__ __forceinline__ void split_adjoint_product(f4 (&acca)[NIBW][CPB], char* __restrict__ STG,
                                                      const char* __restrict__ R, int rld,
                                                      const Raw (&wreg)[NIBW][KC], const char* next, int bytes,
                                                      int lane) {
  if (next) async_copy(STG, next, bytes);
#pragma unroll
  for (int q = 0; q < NIBW; ++q)
#pragma unroll
    for (int cb = 0; cb < CPB; ++cb) acca[q][cb] = f4{0.f, 0.f, 0.f, 0.f};
  // the A fragment of cp block cb for chunk kc + 1 is read as soon as the products of chunk
  // kc that use it have issued; per accumulator the order of Prec::mma is kept
  Raw a[CPB];
#pragma unroll
  for (int cb = 0; cb < CPB; ++cb) a[cb] = Tile<PREC>::load(R, rld, cb, 0, lane);
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
#pragma unroll
    for (int cb = 0; cb < CPB; ++cb) {
#pragma unroll
      for (int q = 0; q < NIBW; ++q) acca[q][cb] = Half<PREC>::mfma(a[cb].b, wreg[q][kc].a, acca[q][cb]);
#pragma unroll
      for (int q = 0; q < NIBW; ++q) acca[q][cb] = Half<PREC>::mfma(a[cb].a, wreg[q][kc].b, acca[q][cb]);
#pragma unroll
      for (int q = 0; q < NIBW; ++q) acca[q][cb] = Half<PREC>::mfma(a[cb].a, wreg[q][kc].a, acca[q][cb]);
      if (kc + 1 < KC) a[cb] = Tile<PREC>::load(R, rld, cb, kc + 1, lane);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // work that waits on vector memory (the pre-activations) stays after the product, so the
  // copy started above runs under it
  __builtin_amdgcn_sched_barrier(0);
}

// Weight-gradient product of the split backward's second role (A operands from the ZT
// tile, B operands in registers), with the copy of the next sub-tile's adjoint into STG
// started first; the restrict qualifiers tell the compiler's wait insertion that the ZT
// reads do not depend on the copy.
template <int PREC, int NOB, int NIBW, int CPB>
__device__ __forceinline__ void split_weight_grad_product(f4 (&accw)[NOB][NIBW], const Raw (&aop)[NIBW][CPB / 2],
                                                          char* __restrict__ STG, const char* __restrict__ ZT,
                                                          const char* next, int bytes, int lane) {
  if (next) async_copy(STG, next, bytes);
  // A operands (one 2 KiB unit per output block) read D blocks ahead of their products, from a
  // ring of D register sets; per accumulator the order of Prec::mma is kept
  constexpr int D = NOB < 3 ? NOB : 3;
#pragma unroll
  for (int cc = 0; cc < CPB / 2; ++cc) {
    Raw u[D];
#pragma unroll
    for (int d = 0; d < D; ++d) u[d] = lds_unit(ZT, d * (CPB / 2) + cc, lane, 64 * 32);
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
      const Raw ao = u[ob % D];
#pragma unroll
      for (int q = 0; q < NIBW; ++q) accw[ob][q] = Half<PREC>::mfma(ao.b, aop[q][cc].a, accw[ob][q]);
#pragma unroll
      for (int q = 0; q < NIBW; ++q) accw[ob][q] = Half<PREC>::mfma(ao.a, aop[q][cc].b, accw[ob][q]);
#pragma unroll
      for (int q = 0; q < NIBW; ++q) accw[ob][q] = Half<PREC>::mfma(ao.a, aop[q][cc].a, accw[ob][q]);
      if (ob + D < NOB) u[ob % D] = lds_unit(ZT, (ob + D) * (CPB / 2) + cc, lane, 64 * 32);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}


}  // namespace pinn
