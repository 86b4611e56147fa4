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
#include "lfsp_device.h"

namespace ldpcfd {

struct DevCode {
  int M, N, E, m;
  const int* row_ptr;      // [M+1]
  const int* e_var;        // [E]
  const int* e_other;      // [E] the other edge of the same variable
  const uint8_t* e_label;  // [E]
  const int* v_edges;      // [N][2] (ascending)
  const uint64_t* colsT;   // [256] byte b of colsT[h] = M_h^T e_b
  const uint8_t* ginv;     // [256]
  const uint8_t* gexp;     // [512]
  const uint16_t* glog;    // [256]
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
// Fourier image of the posterior up to a positive factor.
template <class G>
__device__ __forceinline__ void decide(const float (&Y)[G::R], float (&Xo)[G::R], float* row, int zl,
                                       uint64_t cols_a, uint64_t cols_b, int& hard, int& fa, int& fb) {
  float A[G::R];
#pragma unroll
  for (int r = 0; r < G::R; ++r) A[r] = Y[r];
  wht<G>(A, zl);
  wht<G>(Xo, zl);
#pragma unroll
  for (int r = 0; r < G::R; ++r) A[r] *= Xo[r];
  wht<G>(A, zl);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < G::R; ++r) row[G::z_of(zl, r)] = A[r];
  __builtin_amdgcn_wave_barrier();
  hard = 0; fa = 0; fb = 0;
#pragma unroll
  for (int i = 0; i < G::LOGQ; ++i) {
    hard |= (row[1 << i] < 0.0f) << i;
    fa |= (row[(cols_a >> (8 * i)) & 0xFF] < 0.0f) << i;
    fb |= (row[(cols_b >> (8 * i)) & 0xFF] < 0.0f) << i;
  }
  __builtin_amdgcn_wave_barrier();
}

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
  float* row = lds + (wave * G::T + fl) * G::QP;
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
  decide<G>(Y1, X1, row, zl, uni64(cd.colsT[h1]), uni64(cd.colsT[h2]), hd, fa, fb2);
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
  float* row = lds + (wave * G::T + fl) * G::QP;
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
      permute<G>(st[j], row, zl, uni64(cd.colsT[h]));
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
      permute<G>(o, row, zl, uni64(cd.colsT[hinv]));
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
template <class G, int KMAX, typename S>
__device__ __forceinline__ void fused_item(const DevCode& cd, const float* __restrict__ llr,
                                           const S* __restrict__ cin, S* __restrict__ cout,
                                           uint8_t* __restrict__ hard, uint8_t* __restrict__ fsw, int f,
                                           bool valid, int c, float* row, int zl, int first, int decide_flag,
                                           int write) {
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
      const int v = uni(cd.e_var[e]);
      const int eo = uni(cd.e_other[e]);
      const int h = uni(cd.e_label[e]);
      float t[G::LOGQ];
      prior_coeffs<G>(llr + ((size_t)f * cd.N + v) * G::LOGQ, t);
      if (first) {
#pragma unroll
        for (int r = 0; r < G::R; ++r) st[j][r] = (r == 0 && zl == 0) ? 1.0f : 0.0f;
      } else {
        load_msg<G, S>(cin + fb + (size_t)eo * G::Q, zl, st[j]);
#pragma unroll
        for (int r = 0; r < G::R; ++r) st[j][r] = gamma_inv(st[j][r]);
      }
      conv_prior<G>(st[j], t);
      if (decide_flag && e < eo) {
        float Xo[G::R];
        load_msg<G, S>(cin + fb + (size_t)e * G::Q, zl, Xo);
#pragma unroll
        for (int r = 0; r < G::R; ++r) Xo[r] = gamma_inv(Xo[r]);
        int hd, fa, fo;
        const int ho = uni(cd.e_label[eo]);
        decide<G>(st[j], Xo, row, zl, uni64(cd.colsT[h]), uni64(cd.colsT[ho]), hd, fa, fo);
        if (valid && zl == 0) {
          hard[(size_t)f * cd.N + v] = (uint8_t)hd;
          fsw[(size_t)f * cd.E + e] = (uint8_t)fa;
          fsw[(size_t)f * cd.E + eo] = (uint8_t)fo;
        }
      }
      normalise_gamma<G>(st[j]);
      permute<G>(st[j], row, zl, uni64(cd.colsT[h]));
#pragma unroll
      for (int r = 0; r < G::R; ++r) {
        smag[r] += __builtin_fabsf(st[j][r]);
        ssgn[r] ^= __float_as_uint(st[j][r]);
      }
    }
  }
  if (!write) return;
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
      permute<G>(o, row, zl, uni64(cd.colsT[hinv]));
      if (valid) store_msg<G, S>(cout + fb + (size_t)e * G::Q, zl, o);
    }
  }
}

// Number of XCDs; workgroups are dispatched to them round-robin.
constexpr int kXcds = 8;

// Grid-stride pass over the active frames.  Frame group g is handled by the
// workgroups of XCD g % 8, so both reads of a message within a pass (as the
// other edge of its variable, and by its own check at the owner visit) come
// from the same XCD's L2.  gridDim.x must be a multiple of 8.
template <class G, int KMAX, typename S>
__global__ __launch_bounds__(256) void k_fused(DevCode cd, const float* __restrict__ llr,
                                               const S* __restrict__ cin, S* __restrict__ cout,
                                               uint8_t* __restrict__ hard, uint8_t* __restrict__ fsw,
                                               const int* __restrict__ alist, const int* __restrict__ nact_p,
                                               int first, int decide_flag, int write) {
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
  float* row = lds + (wave * G::T + fl) * G::QP;
  for (long it = (long)(blockIdx.x / kXcds) * waves + wave; it < items; it += stride) {
    const int g = xcd + kXcds * (int)(it / cd.M);
    const int c = (int)(it % cd.M);
    const int slot = g * G::T + fl;
    const bool valid = slot < nact;
    const int f = alist[valid ? slot : nact - 1];
    fused_item<G, KMAX, S>(cd, llr, cin, cout, hard, fsw, f, valid, c, row, zl, first, decide_flag, write);
  }
}

// Syndromes of the tentative decision, one workgroup per active frame: the
// frame's hard decisions and per-edge Fourier sign words are staged in LDS
// (coalesced), then each thread forms checks c = tid, tid + 256, ...:
// direct s_c = sum_{v in V_c} h_cv x^_v and the Fourier word = XOR of the
// check's edge words (edges of a check are contiguous).  unsat[f] / mism[f]
// are set to whether any check is nonzero / any pair differs.
__global__ __launch_bounds__(256) void k_syndrome_frames(DevCode cd, const uint8_t* __restrict__ hard,
                                                         const uint8_t* __restrict__ fsw,
                                                         uint8_t* __restrict__ synd, uint8_t* __restrict__ fsynd,
                                                         uint32_t* __restrict__ unsat, uint32_t* __restrict__ mism,
                                                         const int* __restrict__ alist,
                                                         const int* __restrict__ nact_p, int F_all,
                                                         const uint32_t* __restrict__ active) {
  extern __shared__ uint8_t sm[];
  uint8_t* sh = sm;            // [N]
  uint8_t* sw = sm + cd.N;     // [E]
  const int nact = nact_p ? *nact_p : F_all;
  for (int slot = blockIdx.x; slot < nact; slot += gridDim.x) {
    const int f = alist ? alist[slot] : slot;
    if (active && !active[f]) continue;  // uniform over the block
    for (int i = threadIdx.x; i < cd.N; i += blockDim.x) sh[i] = hard[(size_t)f * cd.N + i];
    for (int i = threadIdx.x; i < cd.E; i += blockDim.x) sw[i] = fsw[(size_t)f * cd.E + i];
    __syncthreads();
    int bad = 0, mm = 0;
    for (int c = threadIdx.x; c < cd.M; c += blockDim.x) {
      const int e0 = cd.row_ptr[c], e1 = cd.row_ptr[c + 1];
      int s = 0, sf = 0;
      for (int e = e0; e < e1; ++e) {
        const int x = sh[cd.e_var[e]];
        if (x) s ^= cd.gexp[cd.glog[cd.e_label[e]] + cd.glog[x]];
        sf ^= sw[e];
      }
      synd[(size_t)f * cd.M + c] = (uint8_t)s;
      if (fsynd) fsynd[(size_t)f * cd.M + c] = (uint8_t)sf;
      bad |= s | sf;
      mm |= s != sf;
    }
    bad = __syncthreads_or(bad);
    mm = __syncthreads_or(mm);
    if (threadIdx.x == 0) {
      unsat[f] = bad ? 1u : 0u;
      mism[f] = mm ? 1u : 0u;
    }
  }
}

// ---------------------------------------------------------------------------
// Syndromes of the tentative decision (one thread per (active frame, check)):
// direct s_c = sum_{v in V_c} h_cv x^_v and Fourier word = XOR of per-edge
// sign words.  Flags the frame when either is nonzero or they differ.
__global__ void k_syndrome(DevCode cd, const uint8_t* __restrict__ hard, const uint8_t* __restrict__ fsw,
                           uint8_t* __restrict__ synd, uint8_t* __restrict__ fsynd,
                           uint32_t* __restrict__ unsat, uint32_t* __restrict__ mism,
                           const int* __restrict__ alist, const int* __restrict__ nact_p, int F_all,
                           const uint32_t* __restrict__ active) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nact = nact_p ? *nact_p : F_all;
  if (i >= (long)nact * cd.M) return;
  const int slot = (int)(i / cd.M), c = (int)(i % cd.M);
  const int f = alist ? alist[slot] : slot;
  if (active && !active[f]) return;
  const int e0 = cd.row_ptr[c], e1 = cd.row_ptr[c + 1];
  int s = 0, sf = 0;
  const int qm1 = (1 << cd.m) - 1;
  for (int e = e0; e < e1; ++e) {
    const int x = hard[(size_t)f * cd.N + cd.e_var[e]];
    const int h = cd.e_label[e];
    if (x) s ^= cd.gexp[(cd.glog[h] + cd.glog[x]) % qm1];
    sf ^= fsw[(size_t)f * cd.E + e];
  }
  synd[(size_t)f * cd.M + c] = (uint8_t)s;
  if (fsynd) fsynd[(size_t)f * cd.M + c] = (uint8_t)sf;
  if (s | sf) atomicOr(&unsat[f], 1u);
  if (s != sf) atomicOr(&mism[f], 1u);
}

// Elementwise conversion between message storage types (n4 groups of 4).
template <typename Sin, typename Sout>
__global__ void k_convert(const Sin* __restrict__ in, Sout* __restrict__ out, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
    float v[4];
    IO<Sin>::load4(in + 4 * i, v);
    IO<Sout>::store4(out + 4 * i, v);
  }
}

__global__ void k_init_frames(int F, uint32_t* active, uint32_t* unsat, uint32_t* mism, int* alist,
                              int* nact, int32_t* iters, uint32_t* status) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f == 0 && nact) *nact = F;
  if (f >= F) return;
  if (active) active[f] = 1u;
  unsat[f] = 0u;
  mism[f] = 0u;
  if (alist) alist[f] = f;
  if (iters) iters[f] = 0;
  if (status) status[f] = 0u;
}

// PLAIN decoder: stopping rule for round ell over all frames.
__global__ void k_retire_plain(int F, int ell, int max_iter, uint32_t* active, uint32_t* unsat,
                               uint32_t* mism, int32_t* iters, uint32_t* status, uint32_t* count) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F || !active[f]) return;
  iters[f] = ell;
  uint32_t st = status[f] | (mism[f] ? 2u : 0u);
  if (!unsat[f]) {
    st |= 1u;
    active[f] = 0u;
  } else if (ell >= max_iter) {
    active[f] = 0u;
  } else {
    atomicAdd(count, 1u);
  }
  status[f] = st;
  unsat[f] = 0u;
  mism[f] = 0u;
}

// FUSED decoder: stopping rule for round ell and stable compaction of the
// active list (single workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_retire_compact(int ell, int max_iter, int* alist, int* tmp,
                                                         int* nact_p, uint32_t* unsat, uint32_t* mism,
                                                         int32_t* iters, uint32_t* status) {
  __shared__ int wsum[16];
  __shared__ int base_s;
  const int nact = *nact_p;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) base_s = 0;
  __syncthreads();
  for (int start = 0; start < nact; start += 1024) {
    const int i = start + tid;
    int keep = 0, f = -1;
    if (i < nact) {
      f = alist[i];
      iters[f] = ell;
      uint32_t st = status[f] | (mism[f] ? 2u : 0u);
      if (!unsat[f]) st |= 1u;
      else if (ell < max_iter) keep = 1;
      status[f] = st;
      unsat[f] = 0u;
      mism[f] = 0u;
    }
    const uint64_t b = __builtin_amdgcn_ballot_w64(keep);
    const int pre = __builtin_popcountll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __builtin_popcountll(b);
    __syncthreads();
    int off = base_s;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (keep) tmp[off + pre] = f;
    __syncthreads();
    if (tid == 0) {
      int s = 0;
      for (int k = 0; k < 16; ++k) s += wsum[k];
      base_s += s;
    }
    __syncthreads();
  }
  const int total = base_s;
  for (int i = tid; i < total; i += 1024) alist[i] = tmp[i];
  __syncthreads();
  if (tid == 0) *nact_p = total;
}

}  // namespace ldpcfd
