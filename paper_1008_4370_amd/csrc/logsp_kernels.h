// The conventional log-domain sum-product decoder (Sec. 2.2), built as the
// comparison the paper makes against the Log-Fourier SP (Table 1): messages
// are log2 pmfs in the probability domain, the check node forms each extrinsic
// message as the XOR convolution of the other k-1 messages (k such
// convolutions per check in Table 1's count; here through forward and backward
// partial convolutions, 3(k-2) pairwise convolutions of q^2 log-sum-exp terms
// in all), and the variable node adds log vectors.  One wavefront per
// (frame, node); symbol x of a vector lives on lane x mod 64 (q/64 symbols per
// lane for q > 64; lanes >= q idle for q < 64).  Log values are clamped to
// [-kLsFloor, 0] after normalisation to max 0.
#pragma once
#include "lfsp_kernels.h"

namespace ldpcfd {

constexpr float kLsFloor = 200.0f;

// Message words of the Log-SP decoder: FP32 log2 probabilities, or 8-bit
// codes k of the log2 probability -k (rounded to nearest, saturating at 255;
// every stored value lies in [-kLsFloor, 0]).
__device__ __forceinline__ float ls_load(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float ls_load(const uint8_t* p, size_t i) { return -(float)p[i]; }
__device__ __forceinline__ void ls_store(float* p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void ls_store(uint8_t* p, size_t i, float v) {
  p[i] = (uint8_t)__builtin_fminf(__builtin_rintf(-v), 255.0f);
}

template <int LOGQ>
struct LsGeo {
  static constexpr int Q = 1 << LOGQ;
  static constexpr int X = Q >= 64 ? Q / 64 : 1;  // symbols per lane
};

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) v = __builtin_fmaxf(v, lane_xor(v, s));
  return v;
}

__device__ __forceinline__ int gf_mul(const DevCode& cd, int a, int x) {
  return (a && x) ? cd.gexp[cd.glog[a] + cd.glog[x]] : 0;
}

// Pairwise convolution of two rows held in the linear domain:
// out(x) = sum_a f(a) g(a ^ x), scaled to maximum 1.  Since f = 2^lf and
// g = 2^lg, log2 out is the log-convolution of lf and lg (log2 sum_a
// 2^(lf(a) + lg(a ^ x))) less its maximum; evaluating it as a sum of products
// of exponentials taken once per entry costs q^2 FMAs instead of q^2
// exponentials.  Both rows have maximum 1, so the sum has a term equal to 1 and
// none above it: nothing overflows, and the scaling keeps every partial
// convolution away from underflow.
//
// Register tiling: a lane owns the four outputs x0..x0+3 (x0 = 4 xb) and one
// of S slices of the a-range, in blocks of four: for a = A + s (A, x0
// multiples of 4) g(a ^ (x0 + r)) = g((A ^ x0) + (s ^ r)), so one 16-byte read
// of f and one of g feed 16 FMAs.  The S partial sums of an output group sit
// on adjacent lanes and are added by XOR shuffles.  f, g, out: LDS rows of Q
// floats, 16-byte aligned (out distinct from f, g).
template <int LOGQ>
__device__ __forceinline__ void ls_conv(const float* f, const float* g, float* out) {
  constexpr int Q = 1 << LOGQ, NB = Q / 4;
  constexpr int S = (256 / Q) < NB ? (256 / Q) : NB;  // slices of the a-range
  constexpr int LANES = NB * S, PER = NB / S;
  const int lane = lane_id();
  const int xb = lane / S, sp = lane % S, x0 = 4 * xb;
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
  if (lane < LANES) {
#pragma unroll 4
    for (int t = 0; t < PER; ++t) {
      const int A = 4 * (sp + S * t);
      const float4 fa = *reinterpret_cast<const float4*>(f + A);
      const float4 ga = *reinterpret_cast<const float4*>(g + (A ^ x0));
      a0 = __builtin_fmaf(fa.x, ga.x, __builtin_fmaf(fa.y, ga.y, __builtin_fmaf(fa.z, ga.z, __builtin_fmaf(fa.w, ga.w, a0))));
      a1 = __builtin_fmaf(fa.x, ga.y, __builtin_fmaf(fa.y, ga.x, __builtin_fmaf(fa.z, ga.w, __builtin_fmaf(fa.w, ga.z, a1))));
      a2 = __builtin_fmaf(fa.x, ga.z, __builtin_fmaf(fa.y, ga.w, __builtin_fmaf(fa.z, ga.x, __builtin_fmaf(fa.w, ga.y, a2))));
      a3 = __builtin_fmaf(fa.x, ga.w, __builtin_fmaf(fa.y, ga.z, __builtin_fmaf(fa.z, ga.y, __builtin_fmaf(fa.w, ga.x, a3))));
    }
  }
#pragma unroll
  for (int o = 1; o < S; o <<= 1) {
    a0 += lane_xor(a0, o);
    a1 += lane_xor(a1, o);
    a2 += lane_xor(a2, o);
    a3 += lane_xor(a3, o);
  }
  const float mx = __builtin_fmaxf(__builtin_fmaxf(a0, a1), __builtin_fmaxf(a2, a3));
  const float sc = __builtin_amdgcn_rcpf(wave_max(mx));
  __syncthreads();
  if (lane < LANES && sp == 0)
    *reinterpret_cast<float4*>(out + x0) = make_float4(a0 * sc, a1 * sc, a2 * sc, a3 * sc);
  __syncthreads();
}

// CHECK TO VARIABLE (Sec. 2.2, Eq. (2)) for the frames alist[0..nf) (frames
// 0..nf-1 when alist is NULL): from the log2
// pmfs v2c[f][e][x] (variable coordinates, maximum 0) to c2v[f][e][x].  The
// incoming rows are exponentiated once on load, the forward/backward partial
// convolutions run on linear rows of maximum 1, and each outgoing row is taken
// back to log2 (less its maximum, floored).  LDS per wavefront (3 kmax + 1) Q
// floats: the label-mapped inputs, the forward and the backward partials, kmax
// rows each, and one output row.
template <int LOGQ, typename M>
__global__ __launch_bounds__(64) void k_logsp_check(DevCode cd, int nf, const int* __restrict__ alist, int kmax,
                                                    const M* __restrict__ v2c, M* __restrict__ c2v) {
  using G = LsGeo<LOGQ>;
  extern __shared__ float ls[];
  float* in = ls;                       // [kmax][Q]
  float* fw = ls + kmax * G::Q;         // [kmax][Q]
  float* bw = ls + 2 * kmax * G::Q;     // [kmax][Q]
  float* ob = ls + 3 * kmax * G::Q;     // [Q]
  const int lane = threadIdx.x;
  const long items = (long)nf * cd.M;
  for (long it = blockIdx.x; it < items; it += gridDim.x) {
    const int fi = (int)(it / cd.M), c = (int)(it % cd.M);
    const int f = alist ? alist[fi] : fi;
    const int e0 = cd.row_ptr[c], deg = cd.row_ptr[c + 1] - e0;
    if (deg == 0) continue;
    // label maps: p~_vc(x) = p_vc(h^-1 x)
    for (int j = 0; j < deg; ++j) {
      const int e = e0 + j;
      const int hinv = cd.ginv[cd.e_label[e]];
      const M* src = v2c + ((size_t)f * cd.E + e) * G::Q;
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        if (x < G::Q) in[j * G::Q + x] = __builtin_amdgcn_exp2f(ls_load(src, gf_mul(cd, hinv, x)));
      }
    }
    __syncthreads();
    // forward partials fw[j] = in[0] (x) ... (x) in[j], backward bw[j] = in[j] (x) ... (x) in[deg-1]
#pragma unroll
    for (int xj = 0; xj < G::X; ++xj) {
      const int x = lane + 64 * xj;
      if (x < G::Q) {
        fw[x] = in[x];
        bw[(deg - 1) * G::Q + x] = in[(deg - 1) * G::Q + x];
      }
    }
    __syncthreads();
    for (int j = 1; j <= deg - 2; ++j) ls_conv<LOGQ>(fw + (j - 1) * G::Q, in + j * G::Q, fw + j * G::Q);
    for (int j = deg - 2; j >= 1; --j) ls_conv<LOGQ>(in + j * G::Q, bw + (j + 1) * G::Q, bw + j * G::Q);
    for (int j = 0; j < deg; ++j) {
      const float* o;
      if (deg == 1) {  // no other edge: the identity of the convolution, mass at 0
#pragma unroll
        for (int xj = 0; xj < G::X; ++xj) {
          const int x = lane + 64 * xj;
          if (x < G::Q) ob[x] = x == 0 ? 1.0f : 0.0f;
        }
        __syncthreads();
        o = ob;
      } else if (j == 0) {
        o = bw + G::Q;
      } else if (j == deg - 1) {
        o = fw + (deg - 2) * G::Q;
      } else {
        ls_conv<LOGQ>(fw + (j - 1) * G::Q, bw + (j + 1) * G::Q, ob);
        o = ob;
      }
      // p_cv(x) = p~_cv(h x), as log2 less the row maximum
      const int e = e0 + j;
      const int h = cd.e_label[e];
      float v[G::X];
      float mx = 0.0f;
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        v[xj] = x < G::Q ? o[gf_mul(cd, h, x)] : 0.0f;
        mx = __builtin_fmaxf(mx, v[xj]);
      }
      const float lmx = __builtin_amdgcn_logf(wave_max(mx));
      M* dst = c2v + ((size_t)f * cd.E + e) * G::Q;
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        if (x < G::Q) ls_store(dst, x, __builtin_fmaxf(__builtin_amdgcn_logf(v[xj]) - lmx, -kLsFloor));
      }
      __syncthreads();
    }
  }
}

// ---- wavefront-per-variable helpers (symbol x on lane x mod 64) -------------

// Walsh-Hadamard transform of a length-Q vector held as p[j] = v(lane + 64 j):
// butterflies over the in-register index, then over lanes (exchanges by DPP
// for lane xor 1, 2, ds_swizzle for 4..16, ds_bpermute for 32; every lane of
// the wavefront takes part).  Lanes >= Q (Q < 64) must hold 0 and keep it.
template <int LOGQ>
__device__ __forceinline__ void wave_wht(float (&p)[LsGeo<LOGQ>::X]) {
  using G = LsGeo<LOGQ>;
  const int lane = lane_id();
#pragma unroll
  for (int hs = 1; hs < G::X; hs <<= 1) {
#pragma unroll
    for (int xj = 0; xj < G::X; ++xj) {
      if (xj & hs) continue;
      const float u = p[xj], w = p[xj + hs];
      p[xj] = u + w;
      p[xj + hs] = u - w;
    }
  }
#pragma unroll
  for (int sh = 1; sh < (G::Q < 64 ? G::Q : 64); sh <<= 1) {
#pragma unroll
    for (int xj = 0; xj < G::X; ++xj) {
      const float o = lane_xor(p[xj], sh);
      p[xj] = (lane & sh) ? o - p[xj] : p[xj] + o;
    }
  }
}

// log2 Pr(X_v = x | y) of the lane's symbols for BPSK LLRs l[0..LOGQ):
// sum_i log2 sigma(t_i), t_i = L_i for bit i of x = 0 and -L_i for 1,
// log2 sigma(t) = -log2(1 + 2^u) with u = -t log2 e.
template <int LOGQ>
__device__ __forceinline__ void log_prior(const float* __restrict__ l, float (&lp)[LsGeo<LOGQ>::X]) {
  using G = LsGeo<LOGQ>;
  const int lane = lane_id();
  float lg[LOGQ];
#pragma unroll
  for (int i = 0; i < LOGQ; ++i) lg[i] = l[i];
#pragma unroll
  for (int xj = 0; xj < G::X; ++xj) {
    const int x = lane + 64 * xj;
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < LOGQ; ++i) {
      const float u = ((x >> i) & 1) ? 1.4426950408889634f * lg[i] : -1.4426950408889634f * lg[i];
      s -= u > 0.0f ? u + __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-u))
                    : __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(u));
    }
    lp[xj] = x < G::Q ? s : -3.0e38f;
  }
}

template <int LOGQ>
__device__ __forceinline__ float row_max(const float (&a)[LsGeo<LOGQ>::X]) {
  float mx = a[0];
#pragma unroll
  for (int xj = 1; xj < LsGeo<LOGQ>::X; ++xj) mx = __builtin_fmaxf(mx, a[xj]);
  return wave_max(mx);
}

// TENTATIVE DECISION from the log2 posterior lp (any offset; -3e38 on lanes >=
// Q): the transform of the linear posterior, then its signs at e_i (the bit
// marginals of x: bitwise-MAP symbol) and at M_h^T e_i for every edge of v
// (the bit marginals of h x: Fourier syndrome words), read from ballots.
template <int LOGQ>
__device__ __forceinline__ void decide_wave(const DevCode& cd, const float (&lp)[LsGeo<LOGQ>::X], int f, int v,
                                            int eb, int ee, uint8_t* __restrict__ hard,
                                            uint8_t* __restrict__ fsw) {
  using G = LsGeo<LOGQ>;
  const int lane = lane_id();
  const float mp = row_max<LOGQ>(lp);
  float p[G::X];
#pragma unroll
  for (int xj = 0; xj < G::X; ++xj) {
    const int x = lane + 64 * xj;
    p[xj] = x < G::Q ? __builtin_amdgcn_exp2f(lp[xj] - mp) : 0.0f;
  }
  wave_wht<LOGQ>(p);
  uint64_t neg[G::X];
#pragma unroll
  for (int xj = 0; xj < G::X; ++xj) neg[xj] = __ballot(p[xj] < 0.0f);
  auto sign_at = [&](int z) {
    uint64_t w = neg[0];
#pragma unroll
    for (int xj = 1; xj < G::X; ++xj)
      if ((z >> 6) == xj) w = neg[xj];
    return (int)((w >> (z & 63)) & 1);
  };
  int hd = 0;
#pragma unroll
  for (int i = 0; i < LOGQ; ++i) hd |= sign_at(1 << i) << i;
  if (lane == 0) hard[(size_t)f * cd.N + v] = (uint8_t)hd;
  for (int k = eb; k < ee; ++k) {
    const int e = cd.v_list[k];
    const uint64_t cm = cd.colsT[cd.e_label[e]];
    int w = 0;
#pragma unroll
    for (int i = 0; i < LOGQ; ++i) w |= sign_at((int)((cm >> (8 * i)) & 0xff)) << i;
    if (lane == 0) fsw[(size_t)f * cd.E + e] = (uint8_t)w;
  }
}

// Signs of the transform of the log2 posterior lp at e_i (bitwise-MAP symbol)
// and at M_h^T e_i for two edges with label maps c1, c2 (colsT words).
template <int LOGQ>
__device__ __forceinline__ void decide_wave2(const float (&lp)[LsGeo<LOGQ>::X], uint64_t c1, uint64_t c2, int& hd,
                                             int& w1, int& w2) {
  using G = LsGeo<LOGQ>;
  const int lane = lane_id();
  const float mp = row_max<LOGQ>(lp);
  float p[G::X];
#pragma unroll
  for (int xj = 0; xj < G::X; ++xj) {
    const int x = lane + 64 * xj;
    p[xj] = x < G::Q ? __builtin_amdgcn_exp2f(lp[xj] - mp) : 0.0f;
  }
  wave_wht<LOGQ>(p);
  uint64_t neg[G::X];
#pragma unroll
  for (int xj = 0; xj < G::X; ++xj) neg[xj] = __ballot(p[xj] < 0.0f);
  auto sign_at = [&](int z) {
    uint64_t w = neg[0];
#pragma unroll
    for (int xj = 1; xj < G::X; ++xj)
      if ((z >> 6) == xj) w = neg[xj];
    return (int)((w >> (z & 63)) & 1);
  };
  hd = w1 = w2 = 0;
#pragma unroll
  for (int i = 0; i < LOGQ; ++i) {
    hd |= sign_at(1 << i) << i;
    w1 |= sign_at((int)((c1 >> (8 * i)) & 0xff)) << i;
    w2 |= sign_at((int)((c2 >> (8 * i)) & 0xff)) << i;
  }
}

// The Log-SP variable node of a weight-2 column, in registers: the message to
// each check is the prior plus the other check's message.
template <int LOGQ, typename M>
__device__ __forceinline__ void logsp_var_w2(const DevCode& cd, int f, int v, int e1, int e2,
                                             const float (&lp)[LsGeo<LOGQ>::X], const M* __restrict__ c2v,
                                             M* __restrict__ v2c, uint8_t* __restrict__ hard,
                                             uint8_t* __restrict__ fsw, int first) {
  using G = LsGeo<LOGQ>;
  const int lane = lane_id();
  const uint64_t c1 = cd.colsT[cd.e_label[e1]], c2 = cd.colsT[cd.e_label[e2]];
  const M* m1 = c2v + ((size_t)f * cd.E + e1) * G::Q;
  const M* m2 = c2v + ((size_t)f * cd.E + e2) * G::Q;
  float a1[G::X], a2[G::X], r1[G::X];
#pragma unroll
  for (int xj = 0; xj < G::X; ++xj) {
    const int x = lane + 64 * xj;
    a1[xj] = a2[xj] = lp[xj];
    r1[xj] = 0.0f;
    if (!first && x < G::Q) {
      r1[xj] = ls_load(m1, x);
      a1[xj] += ls_load(m2, x);  // to the check of e1: the prior and the message from the check of e2
      a2[xj] += r1[xj];
    }
  }
  const float mx1 = row_max<LOGQ>(a1), mx2 = row_max<LOGQ>(a2);
#pragma unroll
  for (int xj = 0; xj < G::X; ++xj) {
    const int x = lane + 64 * xj;
    if (x < G::Q) {
      ls_store(v2c, ((size_t)f * cd.E + e1) * G::Q + x, __builtin_fmaxf(a1[xj] - mx1, -kLsFloor));
      ls_store(v2c, ((size_t)f * cd.E + e2) * G::Q + x, __builtin_fmaxf(a2[xj] - mx2, -kLsFloor));
    }
  }
  if (first) return;
  float post[G::X];
#pragma unroll
  for (int xj = 0; xj < G::X; ++xj) post[xj] = a1[xj] + r1[xj];
  int hd, w1, w2;
  decide_wave2<LOGQ>(post, c1, c2, hd, w1, w2);
  if (lane == 0) {
    hard[(size_t)f * cd.N + v] = (uint8_t)hd;
    fsw[(size_t)f * cd.E + e1] = (uint8_t)w1;
    fsw[(size_t)f * cd.E + e2] = (uint8_t)w2;
  }
}

// VARIABLE TO CHECK and TENTATIVE DECISION (Sec. 2.2) of the Log-SP decoder,
// any column weight j <= 16, for the frames listed as for the check node.
// With first != 0 the message to each check is the prior (round 0, no
// decision); otherwise the message to check c is the prior plus the messages
// from the other checks of v (log domain: a sum), maximum 0, floored, and the
// posterior (prior plus all messages) gives the decision.  LDS per wavefront:
// the j incoming rows (jmax rows of Q floats).
template <int LOGQ, typename M>
__global__ __launch_bounds__(64) void k_logsp_var(DevCode cd, int nf, const int* __restrict__ alist,
                                                  const float* __restrict__ llr, const M* __restrict__ c2v,
                                                  M* __restrict__ v2c, uint8_t* __restrict__ hard,
                                                  uint8_t* __restrict__ fsw, int first) {
  using G = LsGeo<LOGQ>;
  extern __shared__ float rows[];  // [jmax][Q]
  const int lane = threadIdx.x;
  const long items = (long)nf * cd.N;
  for (long it = blockIdx.x; it < items; it += gridDim.x) {
    const int fi = (int)(it / cd.N), v = (int)(it % cd.N);
    const int f = alist ? alist[fi] : fi;
    const int eb = cd.v_ptr[v], ee = cd.v_ptr[v + 1];
    float lp[G::X];
    log_prior<LOGQ>(llr + ((size_t)f * cd.N + v) * LOGQ, lp);
    if (ee - eb == 2) {  // the (2,k) codes: registers only
      logsp_var_w2<LOGQ, M>(cd, f, v, cd.v_list[eb], cd.v_list[eb + 1], lp, c2v, v2c, hard, fsw, first);
      continue;
    }
    if (first) {
      const float mx = row_max<LOGQ>(lp);
      for (int k = eb; k < ee; ++k) {
        M* dst = v2c + ((size_t)f * cd.E + cd.v_list[k]) * G::Q;
#pragma unroll
        for (int xj = 0; xj < G::X; ++xj) {
          const int x = lane + 64 * xj;
          if (x < G::Q) ls_store(dst, x, __builtin_fmaxf(lp[xj] - mx, -kLsFloor));
        }
      }
      continue;
    }
    for (int k = eb; k < ee; ++k) {
      const M* src = c2v + ((size_t)f * cd.E + cd.v_list[k]) * G::Q;
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        if (x < G::Q) rows[(k - eb) * G::Q + x] = ls_load(src, x);
      }
    }
    __syncthreads();
    for (int k = eb; k < ee; ++k) {
      float a[G::X];
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        a[xj] = lp[xj];
        if (x < G::Q)
          for (int s = eb; s < ee; ++s)
            if (s != k) a[xj] += rows[(s - eb) * G::Q + x];
      }
      const float mx = row_max<LOGQ>(a);
      M* dst = v2c + ((size_t)f * cd.E + cd.v_list[k]) * G::Q;
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        if (x < G::Q) ls_store(dst, x, __builtin_fmaxf(a[xj] - mx, -kLsFloor));
      }
    }
    float post[G::X];
#pragma unroll
    for (int xj = 0; xj < G::X; ++xj) {
      const int x = lane + 64 * xj;
      post[xj] = lp[xj];
      if (x < G::Q)
        for (int s = eb; s < ee; ++s) post[xj] += rows[(s - eb) * G::Q + x];
    }
    decide_wave<LOGQ>(cd, post, f, v, eb, ee, hard, fsw);
    __syncthreads();  // rows are rewritten by the next item
  }
}

// VARIABLE TO CHECK and TENTATIVE DECISION of the Log-Fourier SP (Sec. 3.2)
// for any column weight j <= 16 (the PLAIN decoder's variable node for codes
// that are not (2,k)): Lambda_vc = Lambda_v^(0) [+] (the [+]-sum of Lambda_c'v
// over the other checks c' of v), normalised to Lambda_vc(0) = (0,0).  The
// j-fold log-convolution runs through the convolution theorem: each incoming
// message is taken to the probability domain (Gamma^-1, then a Hadamard
// transform), the channel pmf and the other messages are multiplied (as sums
// of log2 values, each clamped at 2^-126), and the product goes back through a
// Hadamard transform and Gamma.  first != 0: Lambda_v^(0)(z) =
// Gamma(prod_{i in z} tanh(L_i / 2)) on every edge.  Same frame list and LDS as
// k_logsp_var; messages in the Log-Fourier word format of the other modes.
// LIN: the linear Fourier SP of Sec. 3.1 instead (messages are P itself,
// normalised to P(0) = 1, no Gamma).
template <int LOGQ, bool LIN>
__global__ __launch_bounds__(64) void k_var_gen(DevCode cd, int nf, const int* __restrict__ alist,
                                                const float* __restrict__ llr, const float* __restrict__ c2v,
                                                float* __restrict__ v2c, uint8_t* __restrict__ hard,
                                                uint8_t* __restrict__ fsw, int first) {
  using G = LsGeo<LOGQ>;
  extern __shared__ float rows[];  // [jmax][Q] log2 of q * p_c'v(x)
  const int lane = threadIdx.x;
  const long items = (long)nf * cd.N;
  for (long it = blockIdx.x; it < items; it += gridDim.x) {
    const int fi = (int)(it / cd.N), v = (int)(it % cd.N);
    const int f = alist ? alist[fi] : fi;
    const int eb = cd.v_ptr[v], ee = cd.v_ptr[v + 1];
    const float* l = llr + ((size_t)f * cd.N + v) * LOGQ;
    if (first) {
      float t[LOGQ];
#pragma unroll
      for (int i = 0; i < LOGQ; ++i) {
        const float x = l[i];
        const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * __builtin_fabsf(x));
        t[i] = __builtin_copysignf((1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e), x);
      }
      float w[G::X];
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int z = lane + 64 * xj;
        float p0 = 1.0f;
#pragma unroll
        for (int i = 0; i < LOGQ; ++i)
          if ((z >> i) & 1) p0 *= t[i];
        w[xj] = LIN ? p0 : gamma_rel(p0, 0.0f);
      }
      for (int k = eb; k < ee; ++k) {
        float* dst = v2c + ((size_t)f * cd.E + cd.v_list[k]) * G::Q;
#pragma unroll
        for (int xj = 0; xj < G::X; ++xj) {
          const int z = lane + 64 * xj;
          if (z < G::Q) dst[z] = w[xj];
        }
      }
      continue;
    }
    float lp[G::X];
    log_prior<LOGQ>(l, lp);
    for (int k = eb; k < ee; ++k) {
      const float* src = c2v + ((size_t)f * cd.E + cd.v_list[k]) * G::Q;
      float p[G::X];
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int z = lane + 64 * xj;
        p[xj] = z < G::Q ? (LIN ? src[z] : gamma_inv(src[z])) : 0.0f;
      }
      wave_wht<LOGQ>(p);
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        if (x < G::Q) rows[(k - eb) * G::Q + x] = __builtin_amdgcn_logf(__builtin_fmaxf(p[xj], 1.17549435e-38f));
      }
    }
    __syncthreads();
    for (int k = eb; k < ee; ++k) {
      float a[G::X];
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        a[xj] = lp[xj];
        if (x < G::Q)
          for (int s = eb; s < ee; ++s)
            if (s != k) a[xj] += rows[(s - eb) * G::Q + x];
      }
      const float mx = row_max<LOGQ>(a);
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int x = lane + 64 * xj;
        a[xj] = x < G::Q ? __builtin_amdgcn_exp2f(a[xj] - mx) : 0.0f;
      }
      wave_wht<LOGQ>(a);
      const float y0 = __builtin_fmaxf(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(a[0]))), 1e-37f);
      const float lg0 = __builtin_amdgcn_logf(y0);
      const float r0 = 1.0f / y0;
      float* dst = v2c + ((size_t)f * cd.E + cd.v_list[k]) * G::Q;
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int z = lane + 64 * xj;
        if (z < G::Q) dst[z] = LIN ? __builtin_fminf(__builtin_fmaxf(a[xj] * r0, -1.0f), 1.0f) : gamma_rel(a[xj], lg0);
      }
    }
    float post[G::X];
#pragma unroll
    for (int xj = 0; xj < G::X; ++xj) {
      const int x = lane + 64 * xj;
      post[xj] = lp[xj];
      if (x < G::Q)
        for (int s = eb; s < ee; ++s) post[xj] += rows[(s - eb) * G::Q + x];
    }
    decide_wave<LOGQ>(cd, post, f, v, eb, ee, hard, fsw);
    __syncthreads();  // rows are rewritten by the next item
  }
}

// M_h^T z for the lane's index z, from cm = colsT[h] (byte b = M_h^T e_b).
template <int LOGQ>
__device__ __forceinline__ int apply_mt(uint64_t cm, int z) {
  int r = 0;
#pragma unroll
  for (int b = 0; b < LOGQ; ++b)
    if ((z >> b) & 1) r ^= (int)((cm >> (8 * b)) & 0xff);
  return r;
}

// CHECK TO VARIABLE of the linear Fourier SP (Sec. 3.1): P~_vc(z) =
// P_vc(M_h^T z); P~_cv(z) = product of P~_v'c(z) over the other edges of the
// check (component-wise, through prefix and suffix products, no division);
// P_cv(z) = P~_cv(M_h^-T z) with M_h^-T = M_{h^-1}^T.  Frames as for
// k_logsp_check; LDS per wavefront 2 kmax Q floats.
template <int LOGQ>
__global__ __launch_bounds__(64) void k_fsp_check(DevCode cd, int nf, const int* __restrict__ alist, int kmax,
                                                  const float* __restrict__ v2c, float* __restrict__ c2v) {
  using G = LsGeo<LOGQ>;
  extern __shared__ float ls[];
  float* in = ls;                // [kmax][Q] check coordinates
  float* out = ls + kmax * G::Q; // [kmax][Q] extrinsic products, check coordinates
  const int lane = threadIdx.x;
  const long items = (long)nf * cd.M;
  for (long it = blockIdx.x; it < items; it += gridDim.x) {
    const int fi = (int)(it / cd.M), c = (int)(it % cd.M);
    const int f = alist ? alist[fi] : fi;
    const int e0 = cd.row_ptr[c], deg = cd.row_ptr[c + 1] - e0;
    for (int j = 0; j < deg; ++j) {
      const int e = e0 + j;
      const uint64_t cm = cd.colsT[cd.e_label[e]];
      const float* src = v2c + ((size_t)f * cd.E + e) * G::Q;
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int z = lane + 64 * xj;
        if (z < G::Q) in[j * G::Q + z] = src[apply_mt<LOGQ>(cm, z)];
      }
    }
    // each lane owns its z in both arrays: no barrier between the passes
#pragma unroll
    for (int xj = 0; xj < G::X; ++xj) {
      const int z = lane + 64 * xj;
      if (z < G::Q) {
        float pre = 1.0f;
        for (int j = 0; j < deg; ++j) {
          out[j * G::Q + z] = pre;
          pre *= in[j * G::Q + z];
        }
        float suf = 1.0f;
        for (int j = deg - 1; j >= 0; --j) {
          out[j * G::Q + z] *= suf;
          suf *= in[j * G::Q + z];
        }
      }
    }
    __syncthreads();
    for (int j = 0; j < deg; ++j) {
      const int e = e0 + j;
      const uint64_t cmi = cd.colsT[cd.ginv[cd.e_label[e]]];
      float* dst = c2v + ((size_t)f * cd.E + e) * G::Q;
#pragma unroll
      for (int xj = 0; xj < G::X; ++xj) {
        const int z = lane + 64 * xj;
        if (z < G::Q) dst[z] = out[j * G::Q + apply_mt<LOGQ>(cmi, z)];
      }
    }
    __syncthreads();
  }
}

}  // namespace ldpcfd
