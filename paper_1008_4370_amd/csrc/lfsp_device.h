// Device building blocks of the Log-Fourier SP decoder (gfx950, wave64).
//
// A message is a length-Q vector (Q = 2^m).  A wavefront holds T = 64/L
// frames; each frame's vector is spread over L consecutive lanes with R = Q/L
// entries per lane.  Entry (lane-in-frame zl, register r) holds index
//     z = (r & 3) | (zl << 2) | ((r >> 2) << (2 + log2 L)),
// so each lane owns runs of 4 consecutive z (one 16-byte FP32 load), z bits
// 0-1 and the high bits live in registers and bits 2..2+log2(L)-1 across the
// frame's lanes.  Butterflies along register bits are plain VALU; along lane
// bits they use DPP quad permutes (lane xor 1, 2), a DPP row rotation (xor 8)
// or ds_swizzle (xor 4, 16).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldpcfd {

// Largest stored magnitude -log2|P| (|P| >= 2^-100 is kept, smaller is 2^-100).
constexpr float kLmax = 100.0f;

template <int LOGQ_, int LOGR_>
struct Geo {
  static constexpr int LOGQ = LOGQ_;
  static constexpr int Q = 1 << LOGQ;
  static constexpr int LOGR = LOGR_;
  static constexpr int R = 1 << LOGR;
  static constexpr int LOGL = LOGQ - LOGR;
  static constexpr int L = 1 << LOGL;
  static constexpr int T = 64 / L;
  // LDS: one row of Q floats per frame (pitch Q, a power of two); entry z of
  // frame fl lives at z ^ swz(fl), which spreads the frames of a wave over the
  // banks and keeps runs of 4 consecutive z contiguous (swz is a multiple of 4).
  static constexpr int QP = Q;
  static __device__ __forceinline__ int swz(int fl) { return (fl << 2) & (Q - 4); }
  static_assert(LOGR >= 2 && LOGL >= 0 && LOGL <= 6, "bad geometry");
  static __host__ __device__ constexpr bool lane_bit(int b) { return b >= 2 && b < 2 + LOGL; }
  static __host__ __device__ constexpr int lane_shift(int b) { return b - 2; }
  static __host__ __device__ constexpr int reg_bit(int b) { return b < 2 ? b : b - LOGL; }
  static __host__ __device__ constexpr int zbit_of_regbit(int rb) { return rb < 2 ? rb : rb + LOGL; }
  static __device__ __forceinline__ int z_of(int zl, int r) {
    return (r & 3) | (zl << 2) | ((r >> 2) << (2 + LOGL));
  }
};

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Value held by lane (this lane xor mask); mask is a compile-time constant
// after unrolling.
__device__ __forceinline__ float lane_xor(float v, int mask) {
  const int iv = __float_as_int(v);
  switch (mask) {
    case 1:
      return __int_as_float(__builtin_amdgcn_mov_dpp(iv, 0xB1, 0xF, 0xF, false));
    case 2:
      return __int_as_float(__builtin_amdgcn_mov_dpp(iv, 0x4E, 0xF, 0xF, false));
    case 4:
      return __int_as_float(__builtin_amdgcn_ds_swizzle(iv, (4 << 10) | 0x1F));
    case 8:
      return __int_as_float(__builtin_amdgcn_ds_swizzle(iv, (8 << 10) | 0x1F));
    case 16:
      return __int_as_float(__builtin_amdgcn_ds_swizzle(iv, (16 << 10) | 0x1F));
    default:
      return __int_as_float(__builtin_amdgcn_ds_bpermute((lane_id() ^ 32) << 2, iv));
  }
}

// v[r] += c * v[r] of lane (this lane xor MASK), for all r: one
// v_fmac_f32_dpp per register for the masks DPP reaches within a row of 16
// lanes (1, 2: quad permutes; 8: a rotation of the row by 8, which is lane
// xor 8), the same single-rounding FMA as the generic form.  A single s_nop 1
// ahead of the block covers the DPP read of a VGPR written by the preceding
// VALU instruction; inside the block every instruction reads a register not
// written earlier in the block.
#define LFD_DPP1 "quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
#define LFD_DPP2 "quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n"
#define LFD_DPP8 "row_ror:8 row_mask:0xf bank_mask:0xf\n"
#define LFD_F(i, c, D) "v_fmac_f32_dpp %" #i ", %" #i ", %" #c " " D
#define LFD_BLK4(c, D) LFD_F(0, c, D) LFD_F(1, c, D) LFD_F(2, c, D) LFD_F(3, c, D)
#define LFD_BLK8(c, D) LFD_BLK4(c, D) LFD_F(4, c, D) LFD_F(5, c, D) LFD_F(6, c, D) LFD_F(7, c, D)
#define LFD_BLK16(c, D)                                                                    \
  LFD_BLK8(c, D) LFD_F(8, c, D) LFD_F(9, c, D) LFD_F(10, c, D) LFD_F(11, c, D) LFD_F(12, c, D) \
  LFD_F(13, c, D) LFD_F(14, c, D) LFD_F(15, c, D)
#define LFD_V4(v) "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3])
#define LFD_V8(v) LFD_V4(v), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7])
#define LFD_V16(v) LFD_V8(v), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), \
                   "+v"(v[13]), "+v"(v[14]), "+v"(v[15])

template <int R>
__device__ __forceinline__ void lane_fmac(float (&v)[R], float c, int mask) {
  if (mask == 1 || mask == 2 || mask == 8) {
    if constexpr (R == 4) {
      if (mask == 1) asm volatile("s_nop 1\n" LFD_BLK4(4, LFD_DPP1) : LFD_V4(v) : "v"(c));
      else if (mask == 2) asm volatile("s_nop 1\n" LFD_BLK4(4, LFD_DPP2) : LFD_V4(v) : "v"(c));
      else asm volatile("s_nop 1\n" LFD_BLK4(4, LFD_DPP8) : LFD_V4(v) : "v"(c));
      return;
    } else if constexpr (R == 8) {
      if (mask == 1) asm volatile("s_nop 1\n" LFD_BLK8(8, LFD_DPP1) : LFD_V8(v) : "v"(c));
      else if (mask == 2) asm volatile("s_nop 1\n" LFD_BLK8(8, LFD_DPP2) : LFD_V8(v) : "v"(c));
      else asm volatile("s_nop 1\n" LFD_BLK8(8, LFD_DPP8) : LFD_V8(v) : "v"(c));
      return;
    } else if constexpr (R == 16) {
      if (mask == 1) asm volatile("s_nop 1\n" LFD_BLK16(16, LFD_DPP1) : LFD_V16(v) : "v"(c));
      else if (mask == 2) asm volatile("s_nop 1\n" LFD_BLK16(16, LFD_DPP2) : LFD_V16(v) : "v"(c));
      else asm volatile("s_nop 1\n" LFD_BLK16(16, LFD_DPP8) : LFD_V16(v) : "v"(c));
      return;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = __builtin_fmaf(c, lane_xor(v[r], mask), v[r]);
}

// Broadcast the value of the frame's first lane (zl = 0) to its L lanes.
template <class G>
__device__ __forceinline__ float bcast_frame0(float v) {
  const int iv = __float_as_int(v);
  if constexpr (G::L == 1) {
    return v;
  } else if constexpr (G::L == 2) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(iv, 0xA0, 0xF, 0xF, false));  // [0,0,2,2]
  } else if constexpr (G::L == 4) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(iv, 0x00, 0xF, 0xF, false));  // [0,0,0,0]
  } else {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((lane_id() & ~(G::L - 1)) << 2, iv));
  }
}

// ---- signed-log map (Sec. 3.2): word = sign bit | -log2|P| --------------------
__device__ __forceinline__ float gamma_inv(float w) {
  const float a = __builtin_amdgcn_exp2f(-__builtin_fabsf(w));
  return __uint_as_float((__float_as_uint(w) & 0x80000000u) | __float_as_uint(a));
}

// Gamma of P / P0 given lg0 = log2(P0) > -inf: magnitude clamped to [0, kLmax].
__device__ __forceinline__ float gamma_rel(float p, float lg0) {
  const float mag = __builtin_amdgcn_fmed3f(lg0 - __builtin_amdgcn_logf(__builtin_fabsf(p)), 0.0f, kLmax);
  return __uint_as_float((__float_as_uint(p) & 0x80000000u) | __float_as_uint(mag));
}

// ---- XOR convolution with the channel prior in the Fourier domain -------------
// The prior of a BPSK symbol is a product over its bits, so its Fourier image is
// P0(z) = prod_{i in z} t_i with t_i = tanh(L_i / 2), and P0 (*) X factors into
// one two-point step per bit: X(z) <- X(z) + t_i X(z xor e_i).
template <class G>
__device__ __forceinline__ void conv_prior(float (&v)[G::R], const float (&t)[G::LOGQ]) {
#pragma unroll
  for (int b = 0; b < G::LOGQ; ++b) {
    const float tb = t[b];
    if (G::lane_bit(b)) {
      lane_fmac<G::R>(v, tb, 1 << G::lane_shift(b));
    } else {
      const int rb = 1 << G::reg_bit(b);
#pragma unroll
      for (int r = 0; r < G::R; ++r) {
        if (!(r & rb)) {
          const float a = v[r], c = v[r | rb];
          v[r] = __builtin_fmaf(tb, c, a);
          v[r | rb] = __builtin_fmaf(tb, a, c);
        }
      }
    }
  }
}

// ---- precise variable-node arithmetic ------------------------------------------
// Near-certain messages have |P(z)| = 1 - delta with delta far below the FP32
// resolution at 1, and reliable channel bits have |t_i| = 1 - u_i likewise.
// Where the channel and the message disagree, the prior convolution cancels
// the leading 1s and leaves a result made of the deltas and u's, which FP32
// values near 1 no longer hold.  The precise form keeps the stored words and
// the check node as they are and runs the variable node in FP64: words are
// widened with 1 - 2^-mu formed from mu directly, the prior factors arrive as
// signed complements c_i = sign(L_i) u_i, the butterflies run in FP64, and the
// normalised magnitude -log2(Y(z)/Y(0)) of a ratio near 1 comes from a series
// in 1 - ratio.

__device__ __forceinline__ double lane_xor_d(double v, int mask) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const float lo = lane_xor(__uint_as_float((uint32_t)u), mask);
  const float hi = lane_xor(__uint_as_float((uint32_t)(u >> 32)), mask);
  return __longlong_as_double((long long)(((unsigned long long)__float_as_uint(hi) << 32) | __float_as_uint(lo)));
}

template <class G>
__device__ __forceinline__ double bcast_frame0_d(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const float lo = bcast_frame0<G>(__uint_as_float((uint32_t)u));
  const float hi = bcast_frame0<G>(__uint_as_float((uint32_t)(u >> 32)));
  return __longlong_as_double((long long)(((unsigned long long)__float_as_uint(hi) << 32) | __float_as_uint(lo)));
}

// sign(w) 2^-|w| in FP64.  For |w| < 1/4, 1 - 2^-|w| = 1 - e^-x (x = |w| ln 2
// < 0.174) is summed as its Taylor series to x^7 (remainder below 1e-9
// relative), so the distance from 1 keeps FP32 relative precision.
__device__ __forceinline__ double gamma_inv_d(float w) {
  const float mu = __builtin_fabsf(w);
  const float x = mu * 0.6931471805599453f;
  float p = __builtin_fmaf(x, 1.0f / 5040.0f, -1.0f / 720.0f);
  p = __builtin_fmaf(x, p, 1.0f / 120.0f);
  p = __builtin_fmaf(x, p, -1.0f / 24.0f);
  p = __builtin_fmaf(x, p, 1.0f / 6.0f);
  p = __builtin_fmaf(x, p, -0.5f);
  p = __builtin_fmaf(x, p, 1.0f);
  const double a = mu < 0.25f ? 1.0 - (double)(x * p) : (double)__builtin_amdgcn_exp2f(-mu);
  return (__float_as_uint(w) & 0x80000000u) ? -a : a;
}

// t = sign(c) (1 - |c|) from a signed complement c.
__device__ __forceinline__ double prior_t_d(float c) {
  const double a = 1.0 - (double)__builtin_fabsf(c);
  return (__float_as_uint(c) & 0x80000000u) ? -a : a;
}

template <class G>
__device__ __forceinline__ void conv_prior_d(double (&v)[G::R], const float (&c)[G::LOGQ]) {
#pragma unroll
  for (int b = 0; b < G::LOGQ; ++b) {
    const double tb = prior_t_d(c[b]);
    if (G::lane_bit(b)) {
      const int mask = 1 << G::lane_shift(b);
#pragma unroll
      for (int r = 0; r < G::R; ++r) v[r] = __builtin_fma(tb, lane_xor_d(v[r], mask), v[r]);
    } else {
      const int rb = 1 << G::reg_bit(b);
#pragma unroll
      for (int r = 0; r < G::R; ++r) {
        if (!(r & rb)) {
          const double a = v[r], d = v[r | rb];
          v[r] = __builtin_fma(tb, d, a);
          v[r | rb] = __builtin_fma(tb, a, d);
        }
      }
    }
  }
}

// Gamma(Y(z) / Y(0)) from FP64 Y: for ratios r >= 15/16, -log2 r =
// (e + e^2/2 + ... + e^7/7) / ln 2 with e = 1 - r (remainder below 4e-9
// relative); below, log2 of r rounded to FP32.  Clamped to [0, kLmax].
template <class G>
__device__ __forceinline__ void normalise_gamma_d(const double (&y)[G::R], float (&out)[G::R]) {
  const double y0 = __builtin_fmax(bcast_frame0_d<G>(y[0]), 1e-300);
  const double inv = 1.0 / y0;
#pragma unroll
  for (int r = 0; r < G::R; ++r) {
    const double rr = __builtin_fabs(y[r]) * inv;
    const float e = (float)(1.0 - rr);
    float s = __builtin_fmaf(e, 1.0f / 7.0f, 1.0f / 6.0f);
    s = __builtin_fmaf(e, s, 1.0f / 5.0f);
    s = __builtin_fmaf(e, s, 1.0f / 4.0f);
    s = __builtin_fmaf(e, s, 1.0f / 3.0f);
    s = __builtin_fmaf(e, s, 0.5f);
    s = __builtin_fmaf(e, s, 1.0f);
    const float near1 = e * s * 1.4426950408889634f;
    const float far = -__builtin_amdgcn_logf((float)rr);
    const float mag = __builtin_amdgcn_fmed3f(rr >= 0.9375 ? near1 : far, 0.0f, kLmax);
    out[r] = __uint_as_float((uint32_t)((unsigned long long)__double_as_longlong(y[r]) >> 32 & 0x80000000ull) |
                             __float_as_uint(mag));
  }
}

// ---- unnormalised Walsh-Hadamard transform, up to a lane sign ----------------
// Returns s(z) V(z) with V(z) = sum_x v(x) (-1)^(z.x) and s(z) = (-1)^popcount(zl)
// (zl = the lane bits of z): along a lane bit each lane forms own +/- partner,
// which is the butterfly output negated on the lanes whose bit is set; the
// flips of later stages factor out because both members of every later pair
// share the bit.  Products of two such transforms carry s(z)^2 = 1.
//
// Lane-reversed input: in a vector held lane-reversed, lane zl of a frame
// holds the entries of lane zl ^ (L - 1), i.e. x'(y) = x(y ^ m) with m the mask
// of the lane bits of the index, and s(z) = (-1)^(z.m).  Then wht_s(x') =
// s(z) sum_y x(y ^ m) (-1)^(z.y) = s(z)^2 V(z) = V(z): the exact transform, with
// no sign to undo.  Loads and LDS gathers produce the reversed layout at no
// cost (the lane's addresses use lane_rev(zl)); the transform's output is in
// the ordinary layout.
template <class G>
__device__ __forceinline__ int lane_rev(int zl) {
  return zl ^ (G::L - 1);
}

template <class G>
__device__ __forceinline__ void wht_s(float (&v)[G::R], int zl) {
#pragma unroll
  for (int b = 0; b < G::LOGQ; ++b) {
    if (G::lane_bit(b)) {
      const int sh = G::lane_shift(b);
      lane_fmac<G::R>(v, ((zl >> sh) & 1) ? -1.0f : 1.0f, 1 << sh);
    } else {
      const int rb = 1 << G::reg_bit(b);
#pragma unroll
      for (int r = 0; r < G::R; ++r) {
        if (!(r & rb)) {
          const float a = v[r], c = v[r | rb];
          v[r] = a + c;
          v[r | rb] = a - c;
        }
      }
    }
  }
}

// ---- label permutation through LDS -------------------------------------------
// out(z) = in(A z) for a GF(2)-linear map A given by its columns col[b] = A e_b
// (a wave-uniform 8-byte word, byte b).  `rb` is the element index of this
// lane's frame row, `cf` the frame's swizzle.  A z = A z_reg ^ A z_lane, so a
// read index is (rb | (A z_lane ^ cf)) ^ A z_reg: one XOR per element with a
// wave-uniform A z_reg.  The values are written from lane zl's entries; the
// read side forms the entries of lane zr (zl, or lane_rev(zl) for a
// lane-reversed result).  Lanes of one frame exchange entries through the row;
// LDS operations of a wave execute in order, and wave barriers keep the
// compiler from moving a lane's accesses across the exchange.
typedef __attribute__((address_space(3))) const float lds_float;

// LDS (address-space 3) byte address of a pointer into shared memory.
__device__ __forceinline__ uint32_t lds_addr(const float* p) {
  return (uint32_t)(size_t)((__attribute__((address_space(3))) const float*)p);
}

template <class G>
__device__ __forceinline__ void lds_put(float* lds, int rb, int cf, int zl, const float (&v)[G::R]) {
#pragma unroll
  for (int h = 0; h < G::R / 4; ++h) {
    const int z0 = (zl << 2) | (h << (2 + G::LOGL));
    *reinterpret_cast<float4*>(lds + (rb | (z0 ^ cf))) = make_float4(v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]);
  }
}

template <class G>
__device__ __forceinline__ void permute(float (&v)[G::R], float* lds, int rb, int cf, int zl, uint64_t cols,
                                       int zr) {
  __builtin_amdgcn_wave_barrier();
  lds_put<G>(lds, rb, cf, zl, v);
  __builtin_amdgcn_wave_barrier();
  int pl = 0;
#pragma unroll
  for (int lb = 0; lb < G::LOGL; ++lb)
    if ((zr >> lb) & 1) pl ^= (int)((cols >> (8 * (2 + lb))) & 0xFF);
  // LDS byte address of the row entry, so each gathered element costs one XOR.
  // Rows start at multiples of 4Q bytes from the array base, which is itself
  // 4Q-aligned (the array is the kernel's only LDS), so XOR-ing an offset
  // below 4Q stays inside the row.  The empty asm keeps the compiler from
  // re-factoring the shift out of the XOR.
  uint32_t lbase4 = lds_addr(lds) + ((uint32_t)(rb | (pl ^ cf)) << 2);
  asm volatile("" : "+v"(lbase4));
#pragma unroll
  for (int r = 0; r < G::R; ++r) {
    uint32_t pr = 0;
#pragma unroll
    for (int rbit = 0; rbit < G::LOGR; ++rbit)
      if ((r >> rbit) & 1) pr ^= (uint32_t)((cols >> (8 * G::zbit_of_regbit(rbit))) & 0xFF);
    v[r] = *reinterpret_cast<const lds_float*>((size_t)(lbase4 ^ (pr << 2)));
  }
  __builtin_amdgcn_wave_barrier();
}

// The gather into the ordinary layout (zr = zl); with zr = lane_rev(zl) the
// result is lane-reversed.
template <class G>
__device__ __forceinline__ void permute(float (&v)[G::R], float* lds, int rb, int cf, int zl, uint64_t cols) {
  permute<G>(v, lds, rb, cf, zl, cols, zl);
}

// ---- message storage ------------------------------------------------------------
struct bf16_t {
  uint16_t bits;
};

template <typename S>
struct IO;
// load_words4 / entry: four entries kept as loaded (32-bit words, 16-bit
// types two to a word) and converted one at a time where they are used, with
// the same conversion as load4; kWords4 words per four entries.
template <>
struct IO<float> {
  static constexpr int kWords4 = 4;
  static __device__ __forceinline__ void load_words4(const float* p, uint32_t* w) {
    const uint4 x = *reinterpret_cast<const uint4*>(p);
    w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
  }
  static __device__ __forceinline__ float entry(const uint32_t* w, int i) { return __uint_as_float(w[i]); }
  static __device__ __forceinline__ void load4(const float* p, float* o) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    o[0] = x.x; o[1] = x.y; o[2] = x.z; o[3] = x.w;
  }
  static __device__ __forceinline__ void store4(float* p, const float* i) {
    *reinterpret_cast<float4*>(p) = make_float4(i[0], i[1], i[2], i[3]);
  }
};
// 16-bit storage holds a different word than FP32: not the signed-log
// Fourier value but the message's pmf scaled by q, q p(x) = sum_z P(z)
// (-1)^(x.z) (the inverse transform of P, clamped at zero; in [0, q] since
// P(0) = 1).  A 16-bit float then keeps every probability to a relative
// precision of 2^-11 (FP16) or 2^-8 (BF16), whereas a 16-bit signed-log
// Fourier word carries P(z) to an absolute ~1e-4, which swamps the small
// probabilities that decide near-certain messages.  The variable node needs
// the pmf anyway (it multiplies the message pmf with the channel pmf), so the
// transform moves from each load to the store of the check node's output.
// FP16 values below 2^-14 are subnormal (q p(x) down to 2^-24 is kept).
template <typename S>
constexpr bool kPmfWords = !__is_same(S, float);
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
template <>
struct IO<_Float16> {
  static constexpr int kWords4 = 2;
  static __device__ __forceinline__ void load_words4(const _Float16* p, uint32_t* w) {
    const uint2 x = *reinterpret_cast<const uint2*>(p);
    w[0] = x.x; w[1] = x.y;
  }
  static __device__ __forceinline__ float entry(const uint32_t* w, int i) {
    const uint16_t b = (uint16_t)((i & 1) ? (w[i >> 1] >> 16) : (w[i >> 1] & 0xFFFFu));
    return (float)__builtin_bit_cast(_Float16, b);
  }
  static __device__ __forceinline__ void load4(const _Float16* p, float* o) {
    const half4_t x = *reinterpret_cast<const half4_t*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = (float)x[i];
  }
  static __device__ __forceinline__ void store4(_Float16* p, const float* i) {
    half4_t x;
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = (_Float16)i[k];
    *reinterpret_cast<half4_t*>(p) = x;
  }
};
__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;  // magnitudes here are finite
}
template <>
struct IO<bf16_t> {
  static constexpr int kWords4 = 2;
  static __device__ __forceinline__ void load_words4(const bf16_t* p, uint32_t* w) {
    const uint2 x = *reinterpret_cast<const uint2*>(p);
    w[0] = x.x; w[1] = x.y;
  }
  static __device__ __forceinline__ float entry(const uint32_t* w, int i) {
    return __uint_as_float((i & 1) ? (w[i >> 1] & 0xFFFF0000u) : (w[i >> 1] << 16));
  }
  static __device__ __forceinline__ void load4(const bf16_t* p, float* o) {
    const uint2 x = *reinterpret_cast<const uint2*>(p);
    o[0] = __uint_as_float(x.x << 16); o[1] = __uint_as_float(x.x & 0xFFFF0000u);
    o[2] = __uint_as_float(x.y << 16); o[3] = __uint_as_float(x.y & 0xFFFF0000u);
  }
  static __device__ __forceinline__ void store4(bf16_t* p, const float* i) {
    uint2 x;
    x.x = f32_to_bf16_rne(i[0]) | (f32_to_bf16_rne(i[1]) << 16);
    x.y = f32_to_bf16_rne(i[2]) | (f32_to_bf16_rne(i[3]) << 16);
    *reinterpret_cast<uint2*>(p) = x;
  }
};

// Load / store one message (this lane's R entries) at `base` = start of the
// frame's Q-vector for one edge.
template <class G, typename S>
__device__ __forceinline__ void load_msg(const S* base, int zl, float (&v)[G::R]) {
#pragma unroll
  for (int h = 0; h < G::R / 4; ++h) IO<S>::load4(base + 4 * zl + 4 * G::L * h, &v[4 * h]);
}
template <class G, typename S>
__device__ __forceinline__ void load_msg_words(const S* base, int zl, uint32_t* w) {
#pragma unroll
  for (int h = 0; h < G::R / 4; ++h) IO<S>::load_words4(base + 4 * zl + 4 * G::L * h, w + IO<S>::kWords4 * h);
}
template <class G, typename S>
__device__ __forceinline__ void store_msg(S* base, int zl, const float (&v)[G::R]) {
#pragma unroll
  for (int h = 0; h < G::R / 4; ++h) IO<S>::store4(base + 4 * zl + 4 * G::L * h, &v[4 * h]);
}

}  // namespace ldpcfd
