// Kernels of the Log-Fourier SP decoder (Kasai & Sakaniwa, Sec. 3.2).
//
// State: check-to-variable messages Lambda_cv (variable coordinates, signed
// log2 words, layout [frame][edge][z]).  The check node applies the label maps
// (Lambda~_vc(z) = Lambda_vc(M_h^T z) and back with M_h^-T), sums sign/magnitude
// over its k edges and forms the extrinsic sums.  The degree-2 variable node
// forms Lambda_vc = Lambda^(0) [+] Lambda_c'v through the convolution theorem:
// the log-convolution with the channel prior is an XOR convolution of Fourier
// vectors, done as one butterfly per bit.  The tentative decision reads the
// signs of the Fourier-domain posterior at alpha^(i-1) and at M_h^T alpha^(i-1).
#pragma once
#include <type_traits>
#include "lfsp_device.h"

namespace ldpcfd {

struct DevCode {
  int M, N, E, m;
  const int* row_ptr;      // [M+1]
  const int* e_var;        // [E]
  const int* e_other;      // [E] the other edge of the same variable (regular codes)
  const uint8_t* e_label;  // [E]
  const int* v_edges;      // [N][2] (ascending; regular codes)
  const uint64_t* colsT;   // [256] byte b of colsT[h] = M_h^T e_b
  const uint8_t* ginv;     // [256]
  const uint8_t* gexp;     // [512]
  const uint16_t* glog;    // [256]
  const uint32_t* e_pack;  // [E] variable | label << 24
  const int* v_ptr;        // [N+1] edges of variable v: v_list[v_ptr[v] .. v_ptr[v+1])
  const int* v_list;       // [E] (ascending per variable)
};

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// t_i = tanh(L_i/2) for the channel LLRs of symbol v of this lane's frame.
template <class G>
__device__ __forceinline__ void prior_coeffs(const float* llr_fv, float (&t)[G::LOGQ]) {
#pragma unroll
  for (int i = 0; i < G::LOGQ; ++i) {
    const float x = llr_fv[i];
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * __builtin_fabsf(x));  // e^-|L|
    const float th = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
    t[i] = __builtin_copysignf(th, x);
  }
}

// Tentative decision from Y = P0 (*) X_c'v and Xo = X_cv (both variable
// coordinates, positive scale irrelevant): Q = WHT(WHT(Y) . WHT(Xo)) is the
// Fourier image of the posterior up to a positive factor.  The lane signs of
// the first two transforms cancel in the product; the third is undone with
// s(z) before the values are written to the frame's LDS row, from which the
// 3m points are read.
// Signs of Q(z) = s(z) A(z) (A as wht_s returns it; A = Q when the
// transform's input was lane-reversed, LANE_SIGNS = false) at the 3m read
// points: e_i (bitwise-MAP bits) and M_h^T e_i for the two edges of the
// variable (cols_a, cols_b), read back through the frame's LDS row.
template <class G, bool LANE_SIGNS = true>
__device__ __forceinline__ void decide_signs(float (&A)[G::R], float* lds, int rb, int cf, int zl, uint64_t cols_a,
                                             uint64_t cols_b, int& hard, int& fa, int& fb) {
  if constexpr (LANE_SIGNS) {
    const float sz = (__builtin_popcount(zl) & 1) ? -1.0f : 1.0f;
#pragma unroll
    for (int r = 0; r < G::R; ++r) A[r] *= sz;
  }
  __builtin_amdgcn_wave_barrier();
  lds_put<G>(lds, rb, cf, zl, A);
  __builtin_amdgcn_wave_barrier();
  hard = 0; fa = 0; fb = 0;
  const int rcf = rb | cf;
#pragma unroll
  for (int i = 0; i < G::LOGQ; ++i) {
    hard |= (lds[rcf ^ (1 << i)] < 0.0f) << i;
    fa |= (lds[rcf ^ (int)((cols_a >> (8 * i)) & 0xFF)] < 0.0f) << i;
    fb |= (lds[rcf ^ (int)((cols_b >> (8 * i)) & 0xFF)] < 0.0f) << i;
  }
  __builtin_amdgcn_wave_barrier();
}

template <class G>
__device__ __forceinline__ void decide(const float (&Y)[G::R], float (&Xo)[G::R], float* lds, int rb, int cf,
                                       int zl, uint64_t cols_a, uint64_t cols_b, int& hard, int& fa, int& fb) {
  float A[G::R];
#pragma unroll
  for (int r = 0; r < G::R; ++r) A[r] = Y[r];
  wht_s<G>(A, zl);
  wht_s<G>(Xo, zl);
#pragma unroll
  for (int r = 0; r < G::R; ++r) A[r] *= Xo[r];
  wht_s<G>(A, zl);
  decide_signs<G>(A, lds, rb, cf, zl, cols_a, cols_b, hard, fa, fb);
}

// The decision from the posterior pmf when the variable node already formed
// pp = p0 . x_c' (the channel pmf times the other message's pmf, clamped):
// the posterior pmf is pp . x_c with x_c the own message's pmf (inverse
// transform of Xo, clamped at zero likewise), one transform back gives Q.
// Two Hadamard transforms instead of three.  Xo is overwritten.
// REV: Xo is held lane-reversed (lane_rev), so its transform carries no lane
// signs.
template <class G, bool REV = false>
__device__ __forceinline__ void decide_pmf(const float (&pp)[G::R], float (&Xo)[G::R], float* lds, int rb, int cf,
                                           int zl, uint64_t cols_a, uint64_t cols_b, int& hard, int& fa, int& fb) {
  const float sz = (!REV && (__builtin_popcount(zl) & 1)) ? -1.0f : 1.0f;
  wht_s<G>(Xo, zl);
#pragma unroll
  for (int r = 0; r < G::R; ++r) Xo[r] = __builtin_fmaxf(REV ? Xo[r] : Xo[r] * sz, 0.0f) * pp[r];
  wht_s<G>(Xo, zl);
  decide_signs<G>(Xo, lds, rb, cf, zl, cols_a, cols_b, hard, fa, fb);
}

// The same decision when the own message arrives as its pmf (16-bit storage,
// kPmfWords): the posterior pmf is pp . xo directly, one transform gives Q.
// pp and xo are held lane-reversed (lane_rev), so Q needs no sign fix.  xo is
// overwritten.
template <class G>
__device__ __forceinline__ void decide_pmf_direct(const float (&pp)[G::R], float (&xo)[G::R], float* lds, int rb,
                                                  int cf, int zl, uint64_t cols_a, uint64_t cols_b, int& hard,
                                                  int& fa, int& fb) {
#pragma unroll
  for (int r = 0; r < G::R; ++r) xo[r] *= pp[r];
  wht_s<G>(xo, zl);
  decide_signs<G, false>(xo, lds, rb, cf, zl, cols_a, cols_b, hard, fa, fb);
}

// ---- tentative decision on the matrix cores ------------------------------------
// For the geometry with 4 lanes per frame (16 frames per wavefront, q = 16, 32,
// 64) the three Hadamard transforms of the decision run as FP16 MFMAs with
// FP32 accumulation: the wave's 16 frames are the N columns of a
// 16x16x16 product, H_q = H_{q/16} (x) H_16 splits into one MFMA with H_16
// per block of 16 entries and a butterfly over the q/16 blocks (VALU, FP32).
// Operand layout of v_mfma_f32_16x16x16f16 (lane l, c = 0..3): A[l % 16][4 (l / 16) + c],
// B[4 (l / 16) + c][l % 16], D[4 (l / 16) + c][l % 16].  A is H_16; a frame's
// vector enters as B through the frame rows in LDS (lane l reads frame l % 16,
// entries 16 b + 4 (l / 16) + c: one 16-byte read per block), and D has the
// layout of B, so the product of two transforms feeds the third directly.
// Inputs are FP16 pairs (hi, lo) holding ~22 bits of each FP32 value; Y is
// scaled to max |Y| = 1 and |Xo| <= 1 make every transform fit, with the
// product scaled by 1/q before the last one.  Only the signs of Q are used.
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ h4_t h16_frag() {
  const int l = lane_id(), i = l & 15, k0 = (l >> 4) << 2;
  h4_t a;
#pragma unroll
  for (int c = 0; c < 4; ++c) a[c] = (__builtin_popcount(i & (k0 + c)) & 1) ? (_Float16)-1.0f : (_Float16)1.0f;
  return a;
}

template <int NB>
__device__ __forceinline__ void wht_blocks(f4_t (&g)[NB]) {
#pragma unroll
  for (int s = 1; s < NB; s <<= 1)
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (!(b & s)) {
        const f4_t x = g[b], y = g[b | s];
        g[b] = x + y;
        g[b | s] = x - y;
      }
}

// An FP32 quadruple as two FP16 operands, x = hi + lo * 2^-11 (lo scaled up
// so that it stays clear of the FP16 subnormal range): H_16 x = H_16 hi +
// 2^-11 H_16 lo keeps about 22 bits of x, with FP32 accumulation.
__device__ __forceinline__ f4_t mfma_h16_split(h4_t H, f4_t x) {
  const f4_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
  h4_t hi, lo;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    hi[c] = (_Float16)x[c];
    lo[c] = (_Float16)((x[c] - (float)hi[c]) * 2048.0f);
  }
  const f4_t a = __builtin_amdgcn_mfma_f32_16x16x16f16(H, hi, zero, 0, 0, 0);
  const f4_t b = __builtin_amdgcn_mfma_f32_16x16x16f16(H, lo, zero, 0, 0, 0);
  return a + b * (1.0f / 2048.0f);
}

// Transform of one LDS-resident vector per frame: H_16 on each block of 16
// entries (read from the frame rows as MFMA B operands, one block at a time to
// keep few registers live), then the butterfly over the blocks.
template <class G>
__device__ __forceinline__ void mfma_wht_rows(const float* lds, int rbn, int cfn, int g4, h4_t H,
                                              f4_t (&t)[G::Q / 16]) {
#pragma unroll
  for (int b = 0; b < G::Q / 16; ++b) {
    const float4 v = *reinterpret_cast<const float4*>(lds + (rbn | ((16 * b + g4) ^ cfn)));
    t[b] = mfma_h16_split(H, f4_t{v.x, v.y, v.z, v.w});
  }
  wht_blocks<G::Q / 16>(t);
}

template <class G>
__device__ __forceinline__ void decide_mfma(const float (&Y)[G::R], const float (&Xo)[G::R], float* lds, int rb,
                                            int cf, int zl, uint64_t cols_a, uint64_t cols_b, int& hard, int& fa,
                                            int& fb) {
  static_assert(G::L == 4 && G::Q >= 16 && G::Q <= 64, "MFMA decision needs 16 frames per wave");
  constexpr int NB = G::Q / 16;
  const int l = lane_id(), n = l & 15, g4 = (l >> 4) << 2;
  // row of frame n of this wave (rows of a wave are T * QP = 16 Q floats apart)
  const int rbn = (rb & ~(G::T * G::QP - 1)) | (n * G::QP), cfn = G::swz(n);
  const h4_t H = h16_frag();
  f4_t ty[NB], tq[NB];
  // Y scaled to max |Y| = 1 over the frame (its 4 lanes form a quad): where
  // the channel and the message disagree all of Y can lie below the FP16
  // range.  Xo needs no scaling (|Xo| <= Xo(0) = 1).
  float ys[G::R];
  float mx = 0.0f;
#pragma unroll
  for (int r = 0; r < G::R; ++r) mx = __builtin_fmaxf(mx, __builtin_fabsf(Y[r]));
  mx = __builtin_fmaxf(mx, lane_xor(mx, 1));
  mx = __builtin_fmaxf(mx, lane_xor(mx, 2));
  const float inv = mx > 0.0f ? 1.0f / mx : 1.0f;
#pragma unroll
  for (int r = 0; r < G::R; ++r) ys[r] = Y[r] * inv;
  __builtin_amdgcn_wave_barrier();
  lds_put<G>(lds, rb, cf, zl, ys);
  __builtin_amdgcn_wave_barrier();
  mfma_wht_rows<G>(lds, rbn, cfn, g4, H, ty);
  __builtin_amdgcn_wave_barrier();
  lds_put<G>(lds, rb, cf, zl, Xo);
  __builtin_amdgcn_wave_barrier();
  mfma_wht_rows<G>(lds, rbn, cfn, g4, H, tq);
  // product (scaled by 1/q to stay in FP16 range), then the third transform
#pragma unroll
  for (int b = 0; b < NB; ++b) tq[b] = mfma_h16_split(H, ty[b] * tq[b] * (1.0f / G::Q));
  wht_blocks<NB>(tq);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int b = 0; b < NB; ++b)
    *reinterpret_cast<float4*>(lds + (rbn | ((16 * b + g4) ^ cfn))) = make_float4(tq[b][0], tq[b][1], tq[b][2], tq[b][3]);
  __builtin_amdgcn_wave_barrier();
  hard = 0; fa = 0; fb = 0;
  const int rcf = rb | cf;
#pragma unroll
  for (int i = 0; i < G::LOGQ; ++i) {
    hard |= (lds[rcf ^ (1 << i)] < 0.0f) << i;
    fa |= (lds[rcf ^ (int)((cols_a >> (8 * i)) & 0xFF)] < 0.0f) << i;
    fb |= (lds[rcf ^ (int)((cols_b >> (8 * i)) & 0xFF)] < 0.0f) << i;
  }
  __builtin_amdgcn_wave_barrier();
}

template <class G>
constexpr bool kMfmaDecision = G::L == 4 && G::Q >= 16 && G::Q <= 64;

// Lambda_vc = Gamma(Y / Y(0)) in place (normalisation P_vc(0) = 1).
template <class G>
__device__ __forceinline__ void normalise_gamma(float (&v)[G::R]) {
  const float y0 = __builtin_fmaxf(bcast_frame0<G>(v[0]), 1e-37f);
  const float lg0 = __builtin_amdgcn_logf(y0);
#pragma unroll
  for (int r = 0; r < G::R; ++r) v[r] = gamma_rel(v[r], lg0);
}

// ---------------------------------------------------------------------------
// PLAIN decoder: variable-node kernel.  One wave = (frame group, variable).
// first != 0: writes the initial messages Lambda_v^(0) to both edges.
// Otherwise: from Lambda_c1v, Lambda_c2v computes Lambda_vc1 = L0 [+] L_c2v,
// Lambda_vc2 = L0 [+] L_c1v and the tentative decision of this round.
template <class G>
__global__ __launch_bounds__(256) void k_var_plain(DevCode cd, int F, const float* __restrict__ llr,
                                                   const float* __restrict__ c2v, float* __restrict__ v2c,
                                                   uint8_t* __restrict__ hard, uint8_t* __restrict__ fsw,
                                                   const uint32_t* __restrict__ active, int first) {
  extern __shared__ float lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long item = (long)blockIdx.x * (blockDim.x >> 6) + wave;
  const int groups = (F + G::T - 1) / G::T;
  if (item >= (long)groups * cd.N) return;
  const int g = (int)(item / cd.N), v = (int)(item % cd.N);
  const int fl = lane / G::L, zl = lane % G::L;
  int f = g * G::T + fl;
  const bool valid = f < F && (active == nullptr || active[f] != 0u);
  if (__builtin_amdgcn_ballot_w64(valid) == 0) return;
  if (f >= F) f = F - 1;
  const int rb = (wave * G::T + fl) * G::QP, cf = G::swz(fl);
  const int e1 = uni(cd.v_edges[2 * v]), e2 = uni(cd.v_edges[2 * v + 1]);
  float t[G::LOGQ];
  prior_coeffs<G>(llr + ((size_t)f * cd.N + v) * G::LOGQ, t);
  const size_t fb = (size_t)f * cd.E * G::Q;
  float Y1[G::R], Y2[G::R];
  if (first) {
#pragma unroll
    for (int r = 0; r < G::R; ++r) Y1[r] = (r == 0 && zl == 0) ? 1.0f : 0.0f;
    conv_prior<G>(Y1, t);
    normalise_gamma<G>(Y1);
    if (valid) {
      store_msg<G, float>(v2c + fb + (size_t)e1 * G::Q, zl, Y1);
      store_msg<G, float>(v2c + fb + (size_t)e2 * G::Q, zl, Y1);
    }
    return;
  }
  float X1[G::R], X2[G::R];
  load_msg<G, float>(c2v + fb + (size_t)e1 * G::Q, zl, X1);
  load_msg<G, float>(c2v + fb + (size_t)e2 * G::Q, zl, X2);
#pragma unroll
  for (int r = 0; r < G::R; ++r) {
    X1[r] = gamma_inv(X1[r]);
    X2[r] = gamma_inv(X2[r]);
    Y1[r] = X2[r];
    Y2[r] = X1[r];
  }
  conv_prior<G>(Y1, t);  // to check c1: prior (*) message from c2
  conv_prior<G>(Y2, t);  // to check c2: prior (*) message from c1
  int hd, fa, fb2;
  const int h1 = uni(cd.e_label[e1]), h2 = uni(cd.e_label[e2]);
  decide<G>(Y1, X1, lds, rb, cf, zl, uni64(cd.colsT[h1]), uni64(cd.colsT[h2]), hd, fa, fb2);
  normalise_gamma<G>(Y1);
  normalise_gamma<G>(Y2);
  if (valid) {
    store_msg<G, float>(v2c + fb + (size_t)e1 * G::Q, zl, Y1);
    store_msg<G, float>(v2c + fb + (size_t)e2 * G::Q, zl, Y2);
    if (zl == 0) {
      hard[(size_t)f * cd.N + v] = (uint8_t)hd;
      fsw[(size_t)f * cd.E + e1] = (uint8_t)fa;
      fsw[(size_t)f * cd.E + e2] = (uint8_t)fb2;
    }
  }
}

// PLAIN decoder: check-node kernel.  One wave = (frame group, check).
// Lambda~_vc(z) = Lambda_vc(M_h^T z); Lambda~_cv = sum over the other edges
// (sign XOR, magnitude add, as total minus own term); Lambda_cv(z) =
// Lambda~_cv(M_h^-T z).
template <class G, int KMAX>
__global__ __launch_bounds__(256) void k_check_plain(DevCode cd, int F, const float* __restrict__ v2c,
                                                     float* __restrict__ c2v,
                                                     const uint32_t* __restrict__ active) {
  extern __shared__ float lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long item = (long)blockIdx.x * (blockDim.x >> 6) + wave;
  const int groups = (F + G::T - 1) / G::T;
  if (item >= (long)groups * cd.M) return;
  const int g = (int)(item / cd.M), c = (int)(item % cd.M);
  const int fl = lane / G::L, zl = lane % G::L;
  int f = g * G::T + fl;
  const bool valid = f < F && (active == nullptr || active[f] != 0u);
  if (__builtin_amdgcn_ballot_w64(valid) == 0) return;
  if (f >= F) f = F - 1;
  const int rb = (wave * G::T + fl) * G::QP, cf = G::swz(fl);
  const int e0 = uni(cd.row_ptr[c]), deg = uni(cd.row_ptr[c + 1]) - e0;
  const size_t fb = (size_t)f * cd.E * G::Q;
  float st[KMAX][G::R];
  float smag[G::R];
  uint32_t ssgn[G::R];
#pragma unroll
  for (int r = 0; r < G::R; ++r) { smag[r] = 0.0f; ssgn[r] = 0u; }
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < deg) {
      const int e = e0 + j;
      const int h = uni(cd.e_label[e]);
      load_msg<G, float>(v2c + fb + (size_t)e * G::Q, zl, st[j]);
      permute<G>(st[j], lds, rb, cf, zl, uni64(cd.colsT[h]));
#pragma unroll
      for (int r = 0; r < G::R; ++r) {
        smag[r] += __builtin_fabsf(st[j][r]);
        ssgn[r] ^= __float_as_uint(st[j][r]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < deg) {
      const int e = e0 + j;
      const int hinv = uni(cd.ginv[cd.e_label[e]]);
      float o[G::R];
#pragma unroll
      for (int r = 0; r < G::R; ++r) {
        const float mag = __builtin_amdgcn_fmed3f(smag[r] - __builtin_fabsf(st[j][r]), 0.0f, kLmax);
        o[r] = __uint_as_float(((ssgn[r] ^ __float_as_uint(st[j][r])) & 0x80000000u) | __float_as_uint(mag));
      }
      permute<G>(o, lds, rb, cf, zl, uni64(cd.colsT[hinv]));
      if (valid) store_msg<G, float>(c2v + fb + (size_t)e * G::Q, zl, o);
    }
  }
}

// ---------------------------------------------------------------------------
// FUSED decoder: one pass per round.  Work item = (group of T active frames,
// check).  For each edge (c, v) the pass rebuilds Lambda_vc = L0 [+] L_c'v from
// the stored state of round l, runs the check node and writes round l+1.  On
// the owner visit of v (the edge with the smaller index) it also forms the
// tentative decision of round l.
//   first:   round 0 -> 1 (Lambda_vc = Lambda^(0), no decision).
//   decide:  form the decision of round l.
//   write:   store round l+1 (off in the last pass).
// Per-frame round state of the fused decoder.  rnd[f] = l is the number of
// check-to-variable rounds computed for frame f; C2V^(l) lives in buffer l & 1.
// A pass on frame f reads C2V^(l) (nothing when l = 0: the variable-to-check
// messages are then Lambda^(0)), forms the tentative decision of round l
// (l >= 1) and writes C2V^(l+1) into buffer (l+1) & 1 unless l has reached the
// frame's max_iter.  Frames at different rounds share a pass.
struct FrameState {
  bool first, decide, write;
  int ell;
};

__device__ __forceinline__ FrameState frame_state(const int* __restrict__ rnd, const int* __restrict__ maxit,
                                                  int maxit_all, int f) {
  FrameState st;
  st.ell = rnd[f];
  const int mi = maxit ? maxit[f] : maxit_all;
  st.first = st.ell == 0;
  st.decide = st.ell >= 1;
  st.write = st.ell < mi;
  return st;
}

// Loads of one edge: the other edge's message, the own message (owner visits
// of a deciding pass) and the prior factors of the variable.  PACK: the two
// messages stay in their storage format (16-bit types two entries to a
// register) until an entry is used, which frees registers for 16-bit storage;
// otherwise they are converted to FP32 as they are loaded.
template <class G, typename S, bool PACK>
struct EdgeLoads;
template <class G, typename S>
struct EdgeLoads<G, S, true> {
  static constexpr int W = G::R / 4 * IO<S>::kWords4;
  uint32_t xw[W];   // incoming message of the variable's other edge
  uint32_t ow[W];   // the edge's own message (decision at the owner visit)
  float l[G::LOGQ];   // prior factors t_i = tanh(L_i / 2) of the variable
  float pr[G::R];     // symbol prior p_v^(0)(x) (arithmetic form kSymbolPrior)
  __device__ __forceinline__ float x(int r) const { return IO<S>::entry(xw + IO<S>::kWords4 * (r >> 2), r & 3); }
  __device__ __forceinline__ float o(int r) const { return IO<S>::entry(ow + IO<S>::kWords4 * (r >> 2), r & 3); }
  __device__ __forceinline__ void load_x(const S* p, int zl) { load_msg_words<G, S>(p, zl, xw); }
  __device__ __forceinline__ void load_o(const S* p, int zl) { load_msg_words<G, S>(p, zl, ow); }
};
template <class G, typename S>
struct EdgeLoads<G, S, false> {
  float xf[G::R];   // as above, converted to FP32 when loaded
  float of[G::R];
  float l[G::LOGQ];
  float pr[G::R];
  __device__ __forceinline__ float x(int r) const { return xf[r]; }
  __device__ __forceinline__ float o(int r) const { return of[r]; }
  __device__ __forceinline__ void load_x(const S* p, int zl) { load_msg<G, S>(p, zl, xf); }
  __device__ __forceinline__ void load_o(const S* p, int zl) { load_msg<G, S>(p, zl, of); }
};

// Arithmetic forms of the variable node: BPSK prior factors in FP32 or FP64,
// a symbol prior pmf per variable (FP32), or the BPSK prior as a pmf formed
// from its bit probabilities (FP32, kProbPrior).
constexpr int kFp32 = 0, kFp64 = 1, kSymbolPrior = 2, kProbPrior = 3;

template <class G, typename S, int AR, bool PACK>
__device__ __forceinline__ void issue_edge(const DevCode& cd, const float* __restrict__ tp, const S* __restrict__ cin,
                                           size_t fb, int f, int e, const FrameState& fs, bool any_decide, int zl,
                                           EdgeLoads<G, S, PACK>& L) {
  const int v = uni(cd.e_var[e]);
  const int eo = uni(cd.e_other[e]);
  if constexpr (AR == kSymbolPrior) {
    load_msg<G, float>(tp + ((size_t)f * cd.N + v) * G::Q, zl, L.pr);
  } else {
    const float* lp = tp + ((size_t)f * cd.N + v) * G::LOGQ;
#pragma unroll
    for (int i = 0; i < G::LOGQ; ++i) L.l[i] = lp[i];
  }
  if (!fs.first) L.load_x(cin + fb + (size_t)eo * G::Q, zl);
  if (any_decide && e < eo && fs.decide) L.load_o(cin + fb + (size_t)e * G::Q, zl);
}

// XOR convolution with a general symbol prior (Sec. 2.1: the channel gives
// Pr(X_v = x | y_v) directly): Y = P0 (*) X is the transform of p0 . x, where x
// is the inverse transform of X, so Y = WHT(p0 . WHT(X)) up to a positive
// factor.  wht_s returns s(z) times the transform, s(z) = (-1)^popcount(zl)
// constant per lane; multiplying by s after each transform removes it.  x is a
// pmf up to that factor, so its negative entries (rounding of near-certain
// messages) are set to zero before the product: in FP32 this removes most of
// the frame errors that the Fourier-domain form adds over the FP64 oracle.
// First half: v := p0 . max(x, 0), x the inverse transform of V (the product
// pmf, up to a positive factor).
// REV: v is held lane-reversed (lane_rev), so its transform carries no lane
// signs; pr and the result are in the ordinary layout.
template <class G, bool REV = false>
__device__ __forceinline__ void symbol_prior_product(float (&v)[G::R], const float (&pr)[G::R], int zl) {
  const float sz = (!REV && (__builtin_popcount(zl) & 1)) ? -1.0f : 1.0f;
  wht_s<G>(v, zl);
#pragma unroll
  for (int r = 0; r < G::R; ++r) v[r] = __builtin_fmaxf(REV ? v[r] : v[r] * sz, 0.0f) * pr[r];
}

// Second half: back to the Fourier domain (REV: v lane-reversed, no sign to
// undo).
template <class G, bool REV = false>
__device__ __forceinline__ void symbol_prior_back(float (&v)[G::R], int zl) {
  wht_s<G>(v, zl);
  if constexpr (!REV) {
    const float sz = (__builtin_popcount(zl) & 1) ? -1.0f : 1.0f;
#pragma unroll
    for (int r = 0; r < G::R; ++r) v[r] *= sz;
  }
}

template <class G>
__device__ __forceinline__ void conv_symbol_prior(float (&v)[G::R], const float (&pr)[G::R], int zl) {
  symbol_prior_product<G>(v, pr, zl);
  symbol_prior_back<G>(v, zl);
}

// The BPSK channel pmf p0(x) = prod_i Pr(b_i = x_i | y) of the lane's entries,
// from the signed complements u_i = sign(L_i) (1 - |tanh(L_i / 2)|): the less
// likely value of bit i has probability |u_i| / 2 = 1 / (1 + e^|L_i|), kept at
// full relative precision, the likelier one 1 - |u_i| / 2.
// Every entry is the product of its m bit factors taken in bit order 0..m-1,
// for every lane geometry, so that every layout gives the same FP32 result.
// The products are formed as a prefix tree in that order: after bit i the
// lane holds one partial product per pattern of the register bits among
// 0..i (the lane bits are fixed per lane), so a lane with R entries spends
// sum_i 2^(register bits <= i) multiplies instead of R (m - 1).
template <class G>
__device__ __forceinline__ void prob_prior(const float (&u)[G::LOGQ], int zl, float (&pr)[G::R]) {
  float p0[G::LOGQ], p1[G::LOGQ];
#pragma unroll
  for (int i = 0; i < G::LOGQ; ++i) {
    const float a = 0.5f * __builtin_fabsf(u[i]);
    const bool zero_likelier = !__builtin_signbit(u[i]);
    p0[i] = zero_likelier ? 1.0f - a : a;
    p1[i] = zero_likelier ? a : 1.0f - a;
  }
  // pr[k] for k < 2^n holds the product over bits 0..i for the register-bit
  // pattern k (register bits numbered in bit order, which is the order of
  // the register index r: see Geo::reg_bit)
  pr[0] = 1.0f;
  int n = 0;
#pragma unroll
  for (int i = 0; i < G::LOGQ; ++i) {
    if (G::lane_bit(i)) {
      const float f = ((zl >> G::lane_shift(i)) & 1) ? p1[i] : p0[i];
#pragma unroll
      for (int k = 0; k < G::R; ++k)
        if (k < (1 << n)) pr[k] *= f;
    } else {
#pragma unroll
      for (int k = G::R - 1; k >= 0; --k)
        if (k < (1 << n)) {
          pr[k | (1 << n)] = pr[k] * p1[i];
          pr[k] *= p0[i];
        }
      ++n;
    }
  }
}

// The check node's output for edge j in check coordinates, total minus own:
// the signed-log word Lambda~_cv (FP32 storage), or, for 16-bit storage
// (kPmfWords), already the linear value Gamma^-1(Lambda~_cv) = sign 2^-mag
// (the map is entrywise, so it may precede the inverse label permutation).
template <typename S, typename Acc>
__device__ __forceinline__ float check_output(Acc smag, uint32_t ssgn, float own) {
  const float mag = __builtin_amdgcn_fmed3f((float)(smag - (Acc)__builtin_fabsf(own)), 0.0f, kLmax);
  const uint32_t sgn = (ssgn ^ __float_as_uint(own)) & 0x80000000u;
  if constexpr (kPmfWords<S>)
    return __uint_as_float(sgn | __float_as_uint(__builtin_amdgcn_exp2f(-mag)));
  else
    return __uint_as_float(sgn | __float_as_uint(mag));
}

// The check node's output (variable coordinates, as check_output forms it) in
// the storage's word format: unchanged for FP32 storage; for 16-bit storage
// the message pmf times q, the transform of P with its negative rounding
// residue set to zero.  For 16-bit storage o arrives lane-reversed (gathered
// with lane_rev, see out_lane), so the transform needs no sign fix, and leaves
// in the ordinary layout.
template <class G, typename S>
__device__ __forceinline__ void to_storage_word(float (&o)[G::R], int zl) {
  if constexpr (kPmfWords<S>) {
    wht_s<G>(o, zl);
#pragma unroll
    for (int r = 0; r < G::R; ++r) o[r] = __builtin_fmaxf(o[r], 0.0f);
  }
}

// Lane whose entries the inverse label permutation gathers into this lane:
// lane-reversed for 16-bit storage (to_storage_word transforms the result).
template <class G, typename S>
__device__ __forceinline__ int out_lane(int zl) {
  return kPmfWords<S> ? lane_rev<G>(zl) : zl;
}

// Lane whose message entries and channel pmf the variable node of the default
// arithmetic (kProbPrior) loads and forms: lane-reversed, so that the first
// transform of each incoming message carries no lane signs (16-bit storage:
// the product pmf's transform back and the decision's transform; FP32
// storage: the transforms of the two loaded Fourier-domain messages).
template <class G, int AR>
__device__ __forceinline__ int in_lane(int zl) {
  return AR == kProbPrior ? lane_rev<G>(zl) : zl;
}

// P (precise): the variable node in FP64 (prior factors given as signed
// complements, see conv_prior_d).
// DM: the decision's transforms on the matrix cores (decide_mfma).
template <class G, int KMAX, typename S, int AR, bool DM>
__device__ __forceinline__ void fused_item(const DevCode& cd, const float* __restrict__ tp, S* __restrict__ buf0,
                                           S* __restrict__ buf1, uint8_t* __restrict__ hard,
                                           uint8_t* __restrict__ fsw, int f, bool valid, const FrameState& fs,
                                           int c, float* lds, int rb, int cf, int zl) {
  static_assert(!kPmfWords<S> || AR == kProbPrior, "16-bit storage (pmf words) takes the default variable node");
  const int e0 = uni(cd.row_ptr[c]), deg = uni(cd.row_ptr[c + 1]) - e0;
  const size_t fb = (size_t)f * cd.E * G::Q;
  const S* cin = (fs.ell & 1) ? buf1 : buf0;
  S* cout = (fs.ell & 1) ? buf0 : buf1;
  const bool any_decide = __builtin_amdgcn_ballot_w64(fs.decide && valid) != 0;
  const bool any_write = __builtin_amdgcn_ballot_w64(fs.write && valid) != 0;
  // some frame of the wave at round 0 (no incoming state): only then the
  // per-entry choice between the initial and the loaded message is needed
  const bool any_first = __builtin_amdgcn_ballot_w64(fs.first) != 0;
  float st[KMAX][G::R];   // Lambda~_vc of each edge (check coordinates)
  // sum of magnitudes over the check's edges (P: FP64, so that a small
  // extrinsic sum next to a large own term survives total minus own)
  constexpr bool P = AR == kFp64;
  using Acc = typename std::conditional<P, double, float>::type;
  Acc smag[G::R];
#pragma unroll
  for (int r = 0; r < G::R; ++r) smag[r] = 0;
  // Edge j+1's loads are in flight while edge j is computed.
  // TWO: two load buffers indexed by the (unrolled, constant) parity of j;
  // the one-buffer form copies the buffer being filled into the one being
  // computed (cur0), about 90 VALU moves per edge in the default arithmetic.
  // TWO is used where the loop unrolls whole and the kernel still compiles
  // without private-memory spills.
  // PACK: 16-bit messages stay packed until use where the loop unrolls whole
  // (KMAX <= 8); with 16 edges the converted form compiles to less private
  // memory.
  constexpr bool TWO = KMAX <= 8 && AR == kProbPrior && (G::LOGQ <= 6 || G::LOGR <= 3);
  constexpr bool PACK = KMAX <= 8;
  EdgeLoads<G, S, PACK> eb[TWO ? 2 : 1];
  const int zx = in_lane<G, AR>(zl);   // lane whose message entries this lane loads
  issue_edge<G, S, AR, PACK>(cd, tp, cin, fb, f, e0, fs, any_decide, zx, eb[0]);
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < deg) {
      const int e = e0 + j;
      const int bc = TWO ? (j & 1) : 0, bn = TWO ? ((j + 1) & 1) : 0;
      const EdgeLoads<G, S, PACK> cur0 = eb[bc];
      const EdgeLoads<G, S, PACK>& cur = TWO ? eb[bc] : cur0;
      if (j + 1 < deg) issue_edge<G, S, AR, PACK>(cd, tp, cin, fb, f, e + 1, fs, any_decide, zx, eb[bn]);
      const int v = uni(cd.e_var[e]);
      const int eo = uni(cd.e_other[e]);
      const int h = uni(cd.e_label[e]);
      float t[G::LOGQ];
#pragma unroll
      for (int i = 0; i < G::LOGQ; ++i) t[i] = cur.l[i];   // prior factors (P, kProbPrior: signed complements)
      double y64[P ? G::R : 1];
      if constexpr (P) {
#pragma unroll
        for (int r = 0; r < G::R; ++r) y64[r] = fs.first ? ((r == 0 && zl == 0) ? 1.0 : 0.0) : gamma_inv_d(cur.x(r));
        conv_prior_d<G>(y64, t);
#pragma unroll
        for (int r = 0; r < G::R; ++r) st[j][r] = (float)y64[r];
      } else if constexpr (kPmfWords<S>) {
        // the stored word is the other message's pmf (times q): the product
        // with the channel pmf needs no transform (both lane-reversed, as
        // the loads)
        float pr[G::R];
        prob_prior<G>(t, zx, pr);
        if (any_first) {
#pragma unroll
          for (int r = 0; r < G::R; ++r) st[j][r] = fs.first ? pr[r] : pr[r] * cur.x(r);
        } else {
#pragma unroll
          for (int r = 0; r < G::R; ++r) st[j][r] = pr[r] * cur.x(r);
        }
        if (any_decide && e < eo) {
          float xo[G::R];
#pragma unroll
          for (int r = 0; r < G::R; ++r) xo[r] = cur.o(r);
          int hd, fa, fo;
          const int ho = uni(cd.e_label[eo]);
          decide_pmf_direct<G>(st[j], xo, lds, rb, cf, zl, uni64(cd.colsT[h]), uni64(cd.colsT[ho]), hd, fa, fo);
          if (valid && fs.decide && zl == 0) {
            hard[(size_t)f * cd.N + v] = (uint8_t)hd;
            fsw[(size_t)f * cd.E + e] = (uint8_t)fa;
            fsw[(size_t)f * cd.E + eo] = (uint8_t)fo;
          }
        }
        symbol_prior_back<G, true>(st[j], zl);
      } else {
#pragma unroll
        for (int r = 0; r < G::R; ++r)
          st[j][r] = fs.first ? ((r == 0 && zx == 0) ? 1.0f : 0.0f) : gamma_inv(cur.x(r));
        if constexpr (AR == kSymbolPrior) {
          conv_symbol_prior<G>(st[j], cur.pr, zl);
        } else if constexpr (AR == kProbPrior) {
          float pr[G::R];
          prob_prior<G>(t, zl, pr);
          symbol_prior_product<G, true>(st[j], pr, zl);   // st[j] loaded lane-reversed
          // owner visit: the decision from the product pmf before the
          // transform back (decide_pmf)
          if (any_decide && e < eo) {
            float xo[G::R];
#pragma unroll
            for (int r = 0; r < G::R; ++r) xo[r] = gamma_inv(cur.o(r));
            int hd, fa, fo;
            const int ho = uni(cd.e_label[eo]);
            decide_pmf<G, true>(st[j], xo, lds, rb, cf, zl, uni64(cd.colsT[h]), uni64(cd.colsT[ho]), hd, fa, fo);
            if (valid && fs.decide && zl == 0) {
              hard[(size_t)f * cd.N + v] = (uint8_t)hd;
              fsw[(size_t)f * cd.E + e] = (uint8_t)fa;
              fsw[(size_t)f * cd.E + eo] = (uint8_t)fo;
            }
          }
          symbol_prior_back<G>(st[j], zl);
        } else {
          conv_prior<G>(st[j], t);
        }
      }
      if (AR != kProbPrior && any_decide && e < eo) {
        float xo[G::R];
#pragma unroll
        for (int r = 0; r < G::R; ++r) xo[r] = gamma_inv(cur.o(r));
        int hd, fa, fo;
        const int ho = uni(cd.e_label[eo]);
        if constexpr (DM)
          decide_mfma<G>(st[j], xo, lds, rb, cf, zl, uni64(cd.colsT[h]), uni64(cd.colsT[ho]), hd, fa, fo);
        else
          decide<G>(st[j], xo, lds, rb, cf, zl, uni64(cd.colsT[h]), uni64(cd.colsT[ho]), hd, fa, fo);
        if (valid && fs.decide && zl == 0) {
          hard[(size_t)f * cd.N + v] = (uint8_t)hd;
          fsw[(size_t)f * cd.E + e] = (uint8_t)fa;
          fsw[(size_t)f * cd.E + eo] = (uint8_t)fo;
        }
      }
      if constexpr (P)
        normalise_gamma_d<G>(y64, st[j]);
      else
        normalise_gamma<G>(st[j]);
      permute<G>(st[j], lds, rb, cf, zl, uni64(cd.colsT[h]));
#pragma unroll
      for (int r = 0; r < G::R; ++r) smag[r] += (Acc)__builtin_fabsf(st[j][r]);
    }
  }
  if (!any_write) return;
  // GF(2) sign of the full sum (XOR over the check's edges)
  uint32_t ssgn[G::R];
#pragma unroll
  for (int r = 0; r < G::R; ++r) ssgn[r] = 0u;
#pragma unroll
  for (int j = 0; j < KMAX; ++j)
    if (j < deg) {
#pragma unroll
      for (int r = 0; r < G::R; ++r) ssgn[r] ^= __float_as_uint(st[j][r]);
    }
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < deg) {
      const int e = e0 + j;
      const int hinv = uni(cd.ginv[cd.e_label[e]]);
      float o[G::R];
#pragma unroll
      for (int r = 0; r < G::R; ++r) o[r] = check_output<S, Acc>(smag[r], ssgn[r], st[j][r]);
      permute<G>(o, lds, rb, cf, zl, uni64(cd.colsT[hinv]), out_lane<G, S>(zl));
      to_storage_word<G, S>(o, zl);
      if (valid && fs.write) store_msg<G, S>(cout + fb + (size_t)e * G::Q, zl, o);
    }
  }
}

// Number of XCDs; workgroups are dispatched to them round-robin.
constexpr int kXcds = 8;

// Grid-stride pass over the active frames.  Frame group g is handled by the
// workgroups of XCD g % 8, so both reads of a message within a pass (as the
// other edge of its variable, and by its own check at the owner visit) come
// from the same XCD's L2.  gridDim.x must be a multiple of 8.
// At least 2 wavefronts per SIMD (<= 256 VGPRs): the stash of a check's
// messages is the largest register consumer.
template <class G, int KMAX, typename S, int AR, bool DM>
__global__ __launch_bounds__(256, 2) void k_fused(DevCode cd, const float* __restrict__ tp, S* __restrict__ buf0,
                                               S* __restrict__ buf1, uint8_t* __restrict__ hard,
                                               uint8_t* __restrict__ fsw, const int* __restrict__ alist,
                                               const int* __restrict__ nact_p, const int* __restrict__ rnd,
                                               const int* __restrict__ maxit, int maxit_all) {
  extern __shared__ float lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int waves = blockDim.x >> 6;
  const int nact = *nact_p;
  const int groups = (nact + G::T - 1) / G::T;
  const int xcd = blockIdx.x % kXcds;
  const long stride = (long)(gridDim.x / kXcds) * waves;
  const long groups_x = (groups - xcd + kXcds - 1) / kXcds;
  const long items = groups_x * cd.M;
  const int fl = lane / G::L, zl = lane % G::L;
  const int rb = (wave * G::T + fl) * G::QP, cf = G::swz(fl);
  for (long it = (long)(blockIdx.x / kXcds) * waves + wave; it < items; it += stride) {
    const int g = xcd + kXcds * (int)(it / cd.M);
    const int c = (int)(it % cd.M);
    const int slot = g * G::T + fl;
    const bool valid = slot < nact;
    const int f = alist[valid ? slot : nact - 1];
    const FrameState fs = frame_state(rnd, maxit, maxit_all, f);
    fused_item<G, KMAX, S, AR, DM>(cd, tp, buf0, buf1, hard, fsw, f, valid, fs, c, lds, rb, cf, zl);
  }
}

// Pass with few active frames: one workgroup of KMAX wavefronts per (group of
// T frames, check), wavefront j taking edge j.  Each computes its
// variable-to-check message (and, on owner visits, the decision) in parallel,
// leaves it in check coordinates in LDS, and after a barrier every wavefront
// sums the check's magnitudes in edge order (the order of fused_item, so the
// results are bit-identical to k_fused) and forms its own extrinsic output.
// A check's latency is then one edge instead of k.  LDS: per wavefront T rows
// of Q floats for the label permutations, and the stash [KMAX][T][Q], whose
// first rows then hold the check's sums.
// HIST (batched retirement): the pass is pass roff of a run of passes between
// two retirements, so a frame is at round rnd[f] + roff; frames past their
// last round do nothing, and the decisions and sign words go to the rows of
// the frame's slot in the active list, hist_hard[slot][N] and
// hist_fsw[slot][E] (the run's pass roff), for the retirement to check.
template <class G, int KMAX, typename S, int AR, bool HIST = false>
__global__ __launch_bounds__(64 * KMAX) void k_fused_split(DevCode cd, const float* __restrict__ tp,
                                                           S* __restrict__ buf0, S* __restrict__ buf1,
                                                           uint8_t* __restrict__ hard, uint8_t* __restrict__ fsw,
                                                           const int* __restrict__ alist,
                                                           const int* __restrict__ nact_p,
                                                           const int* __restrict__ rnd,
                                                           const int* __restrict__ maxit, int maxit_all, int roff,
                                                           uint8_t* __restrict__ hist_hard,
                                                           uint8_t* __restrict__ hist_fsw) {
  extern __shared__ float lds[];
  float* stash = lds + KMAX * G::T * G::QP;
  const int j = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nact = *nact_p;
  const int groups = (nact + G::T - 1) / G::T;
  const long items = (long)groups * cd.M;
  const int fl = lane / G::L, zl = lane % G::L;
  const int rb = (j * G::T + fl) * G::QP, cf = G::swz(fl);
  static_assert(!kPmfWords<S> || AR == kProbPrior, "16-bit storage (pmf words) takes the default variable node");
  constexpr bool P = AR == kFp64;
  using Acc = typename std::conditional<P, double, float>::type;
  for (long it = blockIdx.x; it < items; it += gridDim.x) {
    const int g = (int)(it / cd.M), c = (int)(it % cd.M);
    const int slot = g * G::T + fl;
    const int f = alist[slot < nact ? slot : nact - 1];
    FrameState fs = frame_state(rnd, maxit, maxit_all, f);
    bool valid = slot < nact;
    if constexpr (HIST) {
      fs.ell += roff;
      const int mi = maxit ? maxit[f] : maxit_all;
      valid = valid && fs.ell <= mi;
      fs.first = fs.ell == 0;
      fs.decide = fs.ell >= 1;
      fs.write = fs.ell < mi;
    }
    // rows of this frame's decisions and sign words (formed where they are
    // written, so that no row pointer stays live across the item)
    auto hrow = [&]() { return HIST ? hist_hard + (size_t)slot * cd.N : hard + (size_t)f * cd.N; };
    auto frow = [&]() { return HIST ? hist_fsw + (size_t)slot * cd.E : fsw + (size_t)f * cd.E; };
    const int e0 = uni(cd.row_ptr[c]), deg = uni(cd.row_ptr[c + 1]) - e0;
    const size_t fb = (size_t)f * cd.E * G::Q;
    const S* cin = (fs.ell & 1) ? buf1 : buf0;
    S* cout = (fs.ell & 1) ? buf0 : buf1;
    const bool any_decide = __builtin_amdgcn_ballot_w64(fs.decide && valid) != 0;
    const bool any_write = __builtin_amdgcn_ballot_w64(fs.write && valid) != 0;
    float st[G::R];
    if (j < deg) {
      const int e = e0 + j;
      EdgeLoads<G, S, true> cur;
      const int zx = in_lane<G, AR>(zl);   // lane whose message entries this lane loads
      issue_edge<G, S, AR, true>(cd, tp, cin, fb, f, e, fs, any_decide, zx, cur);
      const int v = uni(cd.e_var[e]);
      const int eo = uni(cd.e_other[e]);
      const int h = uni(cd.e_label[e]);
      float t[G::LOGQ];
#pragma unroll
      for (int i = 0; i < G::LOGQ; ++i) t[i] = cur.l[i];
      double y64[P ? G::R : 1];
      if constexpr (P) {
#pragma unroll
        for (int r = 0; r < G::R; ++r) y64[r] = fs.first ? ((r == 0 && zl == 0) ? 1.0 : 0.0) : gamma_inv_d(cur.x(r));
        conv_prior_d<G>(y64, t);
#pragma unroll
        for (int r = 0; r < G::R; ++r) st[r] = (float)y64[r];
      } else if constexpr (kPmfWords<S>) {
        float pr[G::R];
        prob_prior<G>(t, zx, pr);   // lane-reversed, as the loads
#pragma unroll
        for (int r = 0; r < G::R; ++r) st[r] = fs.first ? pr[r] : pr[r] * cur.x(r);
        if (any_decide && e < eo) {
          float xo[G::R];
#pragma unroll
          for (int r = 0; r < G::R; ++r) xo[r] = cur.o(r);
          int hd, fa, fo;
          const int ho = uni(cd.e_label[eo]);
          decide_pmf_direct<G>(st, xo, lds, rb, cf, zl, uni64(cd.colsT[h]), uni64(cd.colsT[ho]), hd, fa, fo);
          if (valid && fs.decide && zl == 0) {
            hrow()[v] = (uint8_t)hd;
            frow()[e] = (uint8_t)fa;
            frow()[eo] = (uint8_t)fo;
          }
        }
        symbol_prior_back<G, true>(st, zl);
      } else {
#pragma unroll
        for (int r = 0; r < G::R; ++r) st[r] = fs.first ? ((r == 0 && zx == 0) ? 1.0f : 0.0f) : gamma_inv(cur.x(r));
        if constexpr (AR == kSymbolPrior) {
          conv_symbol_prior<G>(st, cur.pr, zl);
        } else if constexpr (AR == kProbPrior) {
          float pr[G::R];
          prob_prior<G>(t, zl, pr);
          symbol_prior_product<G, true>(st, pr, zl);   // st loaded lane-reversed
          if (any_decide && e < eo) {
            float xo[G::R];
#pragma unroll
            for (int r = 0; r < G::R; ++r) xo[r] = gamma_inv(cur.o(r));
            int hd, fa, fo;
            const int ho = uni(cd.e_label[eo]);
            decide_pmf<G, true>(st, xo, lds, rb, cf, zl, uni64(cd.colsT[h]), uni64(cd.colsT[ho]), hd, fa, fo);
            if (valid && fs.decide && zl == 0) {
              hrow()[v] = (uint8_t)hd;
              frow()[e] = (uint8_t)fa;
              frow()[eo] = (uint8_t)fo;
            }
          }
          symbol_prior_back<G>(st, zl);
        } else {
          conv_prior<G>(st, t);
        }
      }
      if (AR != kProbPrior && any_decide && e < eo) {
        float xo[G::R];
#pragma unroll
        for (int r = 0; r < G::R; ++r) xo[r] = gamma_inv(cur.o(r));
        int hd, fa, fo;
        const int ho = uni(cd.e_label[eo]);
        decide<G>(st, xo, lds, rb, cf, zl, uni64(cd.colsT[h]), uni64(cd.colsT[ho]), hd, fa, fo);
        if (valid && fs.decide && zl == 0) {
          hrow()[v] = (uint8_t)hd;
          frow()[e] = (uint8_t)fa;
          frow()[eo] = (uint8_t)fo;
        }
      }
      if constexpr (P)
        normalise_gamma_d<G>(y64, st);
      else
        normalise_gamma<G>(st);
      permute<G>(st, lds, rb, cf, zl, uni64(cd.colsT[h]));
      lds_put<G>(stash, rb, cf, zl, st);
    }
    __syncthreads();
    // The check's sums, once per workgroup: every thread takes a share of the
    // stash entries and adds the magnitudes (XORs the sign words) over the
    // edges in edge order, as fused_item does, so the sums are bit-identical.
    // They replace the stash in place: entry x of stash rows 0, 1 (and 2)
    // takes the magnitude's (low) word, the sign word (and the FP64
    // magnitude's high word); only the thread of entry x touches them.  The
    // frames of a workgroup are the same for all its wavefronts, so any_write
    // is uniform over the workgroup.
    constexpr int TQ = G::T * G::QP;
    static_assert(KMAX >= 3, "the sums take stash rows 0..2");
    uint32_t* su = reinterpret_cast<uint32_t*>(stash);
    if (any_write) {
      for (int x = threadIdx.x; x < TQ; x += blockDim.x) {
        Acc m = 0;
        uint32_t sg = 0u;
        for (int i = 0; i < deg; ++i) {
          const float w = stash[i * TQ + x];
          m += (Acc)__builtin_fabsf(w);
          sg ^= __float_as_uint(w);
        }
        if constexpr (P) {
          const uint64_t mb = (uint64_t)__double_as_longlong(m);
          su[x] = (uint32_t)mb;
          su[2 * TQ + x] = (uint32_t)(mb >> 32);
        } else {
          su[x] = __float_as_uint(m);
        }
        su[TQ + x] = sg;
      }
    }
    __syncthreads();
    if (j < deg && any_write) {
      Acc smag[G::R];
      uint32_t ssgn[G::R];
#pragma unroll
      for (int h4 = 0; h4 < G::R / 4; ++h4) {
        const int x = fl * G::QP + (((zl << 2) | (h4 << (2 + G::LOGL))) ^ cf);
        const uint4 lo = *reinterpret_cast<const uint4*>(su + x);
        const uint4 sg = *reinterpret_cast<const uint4*>(su + TQ + x);
        const uint32_t l4[4] = {lo.x, lo.y, lo.z, lo.w};
        const uint32_t s4[4] = {sg.x, sg.y, sg.z, sg.w};
        uint32_t h4w[4] = {0u, 0u, 0u, 0u};
        if constexpr (P) {
          const uint4 hi = *reinterpret_cast<const uint4*>(su + 2 * TQ + x);
          h4w[0] = hi.x;
          h4w[1] = hi.y;
          h4w[2] = hi.z;
          h4w[3] = hi.w;
        }
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          ssgn[4 * h4 + q4] = s4[q4];
          if constexpr (P)
            smag[4 * h4 + q4] = __longlong_as_double((long long)(((uint64_t)h4w[q4] << 32) | l4[q4]));
          else
            smag[4 * h4 + q4] = __uint_as_float(l4[q4]);
        }
      }
      const int e = e0 + j;
      const int hinv = uni(cd.ginv[cd.e_label[e]]);
      float o[G::R];
#pragma unroll
      for (int r = 0; r < G::R; ++r) o[r] = check_output<S, Acc>(smag[r], ssgn[r], st[r]);
      permute<G>(o, lds, rb, cf, zl, uni64(cd.colsT[hinv]), out_lane<G, S>(zl));
      to_storage_word<G, S>(o, zl);
      if (valid && fs.write) store_msg<G, S>(cout + fb + (size_t)e * G::Q, zl, o);
    }
    __syncthreads();  // the stash is rewritten by the next item
  }
}

}  // namespace ldpcfd
