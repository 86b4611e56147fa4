// Per-frame kernels of the decoders that do not depend on the field size:
// initial state, prior factors, syndromes, stopping rule and compaction,
// storage conversion and emulated low-bit storage.  Included by the host
// translation unit only (the field-size templated kernels live in
// lfsp_kernels.h / logsp_kernels.h and are instantiated per field size).
#pragma once
#include "lfsp_kernels.h"

namespace ldpcfd {

// Syndromes of the tentative decision, for codes whose rows do not fit in LDS
// (one thread per (active frame, check)): direct s_c = sum_{v in V_c} h_cv x^_v
// and Fourier word = XOR of per-edge sign words.  Flags the frame when either
// is nonzero or they differ (unsat / mism must be zero on entry).
__global__ void k_syndrome(DevCode cd, const uint8_t* __restrict__ hard, const uint8_t* __restrict__ fsw,
                           uint8_t* __restrict__ synd, uint8_t* __restrict__ fsynd,
                           uint32_t* __restrict__ unsat, uint32_t* __restrict__ mism,
                           const int* __restrict__ alist, const int* __restrict__ nact_p, int F_all,
                           const uint32_t* __restrict__ active, const int* __restrict__ rnd) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nact = nact_p ? *nact_p : F_all;
  if (i >= (long)nact * cd.M) return;
  const int slot = (int)(i / cd.M), c = (int)(i % cd.M);
  const int f = alist ? alist[slot] : slot;
  if (active && !active[f]) return;
  if (rnd && rnd[f] == 0) return;
  const int e0 = cd.row_ptr[c], e1 = cd.row_ptr[c + 1];
  int s = 0, sf = 0;
  for (int e = e0; e < e1; ++e) {
    const int x = hard[(size_t)f * cd.N + cd.e_var[e]];
    if (x) s ^= cd.gexp[cd.glog[cd.e_label[e]] + cd.glog[x]];
    sf ^= fsw[(size_t)f * cd.E + e];
  }
  synd[(size_t)f * cd.M + c] = (uint8_t)s;
  if (fsynd) fsynd[(size_t)f * cd.M + c] = (uint8_t)sf;
  if (s | sf) atomicOr(&unsat[f], 1u);
  if (s != sf) atomicOr(&mism[f], 1u);
}

// INITIALIZATION (Sec. 3.2): the initial message Lambda_v^(0) is Gamma of the
// Fourier transform of the channel pmf, which for BPSK factors over the bits:
// P_v^(0)(z) = prod_{i in z} tanh(L_{v,i}/2).  The passes keep only these m
// factors per symbol (the same 4 N m bytes as the LLRs) and apply them as the
// prior convolution; this kernel forms them once per decode.
// comp != 0: the signed complement sign(L) (1 - |tanh(L/2)|) = sign(L) 2 e / (1 + e)
// instead (precise variable node), exact in FP32 relative precision for reliable bits.
__device__ __forceinline__ float prior_factor(float x, int comp) {
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * __builtin_fabsf(x));  // e^-|L|
  return __builtin_copysignf((comp ? 2.0f * e : 1.0f - e) / (1.0f + e), x);
}

__global__ void k_prior_factors(const float* __restrict__ llr, float* __restrict__ t, size_t n, int comp) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    t[i] = prior_factor(llr[i], comp);
}

// Syndromes of the tentative decision, one workgroup per active frame: the
// frame's hard decisions and per-edge Fourier sign words are staged in LDS
// (word loads when the rows are word aligned), the field tables once per
// workgroup; each thread then forms checks c = tid, tid + 256, ...: direct
// s_c = sum_{v in V_c} h_cv x^_v and the Fourier word = XOR of the check's
// edge words (edges of a check are contiguous).  unsat[f] / mism[f] are set to
// whether any check is nonzero / any pair differs.
__device__ __forceinline__ void syndrome_frames_body(const DevCode& cd, const uint8_t* __restrict__ hard,
                                                     const uint8_t* __restrict__ fsw, uint8_t* __restrict__ synd,
                                                     uint8_t* __restrict__ fsynd, uint32_t* __restrict__ unsat,
                                                     uint32_t* __restrict__ mism, const int* __restrict__ alist,
                                                     int nact, const uint32_t* __restrict__ active,
                                                     const int* __restrict__ rnd, uint32_t* smw, uint8_t* s_exp,
                                                     uint16_t* s_log) {
  uint8_t* sh = reinterpret_cast<uint8_t*>(smw);   // [N] (rounded up to words)
  const int nw = (cd.N + 3) >> 2, ew = (cd.E + 3) >> 2;
  uint8_t* sw = reinterpret_cast<uint8_t*>(smw + nw);  // [E]
  for (int i = threadIdx.x; i < 512; i += blockDim.x) s_exp[i] = cd.gexp[i];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) s_log[i] = cd.glog[i];
  const bool wN = (cd.N & 3) == 0, wE = (cd.E & 3) == 0;
  for (int slot = blockIdx.x; slot < nact; slot += gridDim.x) {
    const int f = alist ? alist[slot] : slot;
    if (active && !active[f]) continue;  // uniform over the block
    if (rnd && rnd[f] == 0) continue;     // fresh frame: no decision this pass
    if (wN) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(hard + (size_t)f * cd.N);
      for (int i = threadIdx.x; i < nw; i += blockDim.x) smw[i] = src[i];
    } else {
      for (int i = threadIdx.x; i < cd.N; i += blockDim.x) sh[i] = hard[(size_t)f * cd.N + i];
    }
    if (wE) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(fsw + (size_t)f * cd.E);
      for (int i = threadIdx.x; i < ew; i += blockDim.x) smw[nw + i] = src[i];
    } else {
      for (int i = threadIdx.x; i < cd.E; i += blockDim.x) sw[i] = fsw[(size_t)f * cd.E + i];
    }
    __syncthreads();
    int bad = 0, mm = 0;
    for (int c = threadIdx.x; c < cd.M; c += blockDim.x) {
      const int e0 = cd.row_ptr[c], e1 = cd.row_ptr[c + 1];
      int s = 0, sf = 0;
      // the row's edges in groups of 8 whose loads are issued together (one
      // memory latency per group, not one per edge); XOR sums in any order
      for (int eb = e0; eb < e1; eb += 8) {
        uint32_t pk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) pk[u] = eb + u < e1 ? cd.e_pack[eb + u] : 0u;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (eb + u < e1) {
            const int x = sh[pk[u] & 0xFFFFFFu];
            if (x) s ^= s_exp[s_log[pk[u] >> 24] + s_log[x]];
            sf ^= sw[eb + u];
          }
        }
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

__global__ __launch_bounds__(256) void k_syndrome_frames(DevCode cd, const uint8_t* __restrict__ hard,
                                                         const uint8_t* __restrict__ fsw,
                                                         uint8_t* __restrict__ synd, uint8_t* __restrict__ fsynd,
                                                         uint32_t* __restrict__ unsat, uint32_t* __restrict__ mism,
                                                         const int* __restrict__ alist,
                                                         const int* __restrict__ nact_p, int F_all,
                                                         const uint32_t* __restrict__ active,
                                                         const int* __restrict__ rnd) {
  extern __shared__ uint32_t smw[];
  __shared__ uint8_t s_exp[512];
  __shared__ uint16_t s_log[256];
  syndrome_frames_body(cd, hard, fsw, synd, fsynd, unsat, mism, alist, nact_p ? *nact_p : F_all, active, rnd, smw,
                       s_exp, s_log);
}

// In-place Hadamard transform of a length-q FP64 vector in LDS by q/2 or
// more threads (q <= blockDim.x).
__device__ __forceinline__ void lds_wht_d(double* a, int q) {
  const int z = threadIdx.x;
  for (int s = 1; s < q; s <<= 1) {
    if (z < q / 2) {
      const int lo = (z / s) * 2 * s + (z % s), hi = lo + s;
      const double a0 = a[lo], a1 = a[hi];
      a[lo] = a0 + a1;
      a[hi] = a0 - a1;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ float load_pmf_word(_Float16 w) { return (float)w; }
__device__ __forceinline__ float load_pmf_word(bf16_t w) { return __uint_as_float((uint32_t)w.bits << 16); }
__device__ __forceinline__ void store_pmf_word(_Float16* p, float v) { *p = (_Float16)v; }
__device__ __forceinline__ void store_pmf_word(bf16_t* p, float v) { p->bits = (uint16_t)f32_to_bf16_rne(v); }

// Signed-log message vectors [nvec][q] (FP32 layout) -> 16-bit pmf words:
// P(z) = sign 2^-|w| in FP64, q p(x) = sum_z P(z) (-1)^(x.z), clamped at zero,
// rounded to FP32 and then to the storage type.
template <typename S>
__global__ void k_lambda_to_pmf(const float* __restrict__ in, S* __restrict__ out, long nvec, int q) {
  extern __shared__ double shd[];
  const int z = threadIdx.x;
  for (long i = blockIdx.x; i < nvec; i += gridDim.x) {
    if (z < q) {
      const float w = in[i * q + z];
      const double a = exp2(-(double)__builtin_fabsf(w));
      shd[z] = (__float_as_uint(w) & 0x80000000u) ? -a : a;
    }
    __syncthreads();
    lds_wht_d(shd, q);
    if (z < q) store_pmf_word(out + i * q + z, (float)(shd[z] > 0.0 ? shd[z] : 0.0));
    __syncthreads();  // shd is rewritten by the next vector
  }
}

// 16-bit pmf words [nvec][q] -> signed-log FP32 words of the same message,
// normalised to P(0) = 1: Q(z) = sum_x (q p(x)) (-1)^(x.z) in FP64, word =
// sign | min(-log2 |Q(z) / Q(0)|, kLmax).
template <typename S>
__global__ void k_pmf_to_lambda(const S* __restrict__ in, float* __restrict__ out, long nvec, int q) {
  extern __shared__ double shd[];
  const int z = threadIdx.x;
  for (long i = blockIdx.x; i < nvec; i += gridDim.x) {
    if (z < q) shd[z] = (double)load_pmf_word(in[i * q + z]);
    __syncthreads();
    lds_wht_d(shd, q);
    if (z < q) {
      const double q0 = shd[0] > 0.0 ? shd[0] : 1e-300;
      const double r = shd[z] / q0;
      const double mag = __builtin_fmin(__builtin_fmax(-log2(__builtin_fabs(r)), 0.0), (double)kLmax);
      const float fm = (float)mag;
      out[i * q + z] = r < 0.0 ? -fm : fm;
    }
    __syncthreads();
  }
}

// Initial per-frame state; nact[2] (the syndrome/retire ticket of the fused
// decoder's workspace) is cleared with the active count.
__global__ void k_init_frames(int F, uint32_t* active, uint32_t* unsat, uint32_t* mism, int* alist,
                              int* nact, int32_t* iters, uint32_t* status, int* rnd, int rnd0) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f == 0 && nact) {
    nact[0] = F;
    nact[2] = 0;
  }
  if (f >= F) return;
  if (rnd) rnd[f] = rnd0;
  if (active) active[f] = 1u;
  unsat[f] = 0u;
  mism[f] = 0u;
  if (alist) alist[f] = f;
  if (iters) iters[f] = 0;
  if (status) status[f] = 0u;
}

// PLAIN and LOGSP decoders: stopping rule for round ell over all frames; with
// alist, the frames that continue are appended to it (in counter order).
// early_stop = 0: frames run to max_iter whatever their syndromes (the
// converged bit then reports the last round's codeword test).
__global__ void k_retire_plain(int F, int ell, int max_iter, uint32_t* active, uint32_t* unsat,
                               uint32_t* mism, int32_t* iters, uint32_t* status, uint32_t* count, int* alist,
                               int early_stop) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F || !active[f]) return;
  iters[f] = ell;
  uint32_t st = status[f] | (mism[f] ? 2u : 0u);
  if (!unsat[f] && (early_stop || ell >= max_iter)) {
    st |= 1u;
    active[f] = 0u;
  } else if (ell >= max_iter) {
    active[f] = 0u;
  } else {
    const uint32_t slot = atomicAdd(count, 1u);
    if (alist) alist[slot] = f;
  }
  status[f] = st;
  unsat[f] = 0u;
  mism[f] = 0u;
}

// FUSED decoder: stopping rule and stable compaction of the active list by one
// workgroup of NT threads.  For each active frame with l = rnd[f] >= 1 the
// decision of round l was formed in the pass: iters = l; the frame stops when
// both syndromes were zero (unless early_stop = 0), or at l = max_iter, with
// the converged bit set when its last decision passed the codeword test.
// Continuing frames advance rnd.  Stopped frames are appended to `done` (when
// given) for harvesting.
template <int NT>
__device__ __forceinline__ void retire_compact_body(int maxit_all, const int* __restrict__ maxit, int early_stop,
                                                    int* alist, int* tmp, int* nact_p, uint32_t* unsat,
                                                    uint32_t* mism, int32_t* iters, uint32_t* status, int* rnd,
                                                    int* done, int* ndone, int* wsum, int* base_s) {
  constexpr int NW = NT / 64;
  const int nact = *nact_p;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) *base_s = 0;
  __syncthreads();
  for (int start = 0; start < nact; start += NT) {
    const int i = start + tid;
    int keep = 0, f = -1, stop = 0;
    if (i < nact) {
      f = alist[i];
      const int ell = rnd[f];
      if (ell >= 1) {
        iters[f] = ell;
        uint32_t st = status[f] | (mism[f] ? 2u : 0u);
        const bool conv = !unsat[f];
        const bool more = ell < (maxit ? maxit[f] : maxit_all);
        keep = more && !(conv && early_stop);
        if (conv && !keep) st |= 1u;
        status[f] = st;
        unsat[f] = 0u;
        mism[f] = 0u;
      } else {
        keep = 1;
      }
      if (keep) rnd[f] = ell + 1;
      stop = !keep;
    }
    if (done && stop) done[atomicAdd(ndone, 1)] = f;
    const uint64_t b = __builtin_amdgcn_ballot_w64(keep);
    const int pre = __builtin_popcountll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __builtin_popcountll(b);
    __syncthreads();
    int off = *base_s;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (keep) tmp[off + pre] = f;
    __syncthreads();
    if (tid == 0) {
      int s2 = 0;
      for (int k = 0; k < NW; ++k) s2 += wsum[k];
      *base_s += s2;
    }
    __syncthreads();
  }
  const int total = *base_s;
  for (int i = tid; i < total; i += NT) alist[i] = tmp[i];
  __syncthreads();
  if (tid == 0) *nact_p = total;
}

// The same as a kernel of one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_retire_compact(int maxit_all, const int* __restrict__ maxit,
                                                         int early_stop, int* alist, int* tmp, int* nact_p,
                                                         uint32_t* unsat, uint32_t* mism, int32_t* iters,
                                                         uint32_t* status, int* rnd, int* done, int* ndone) {
  __shared__ int wsum[16];
  __shared__ int base_s;
  retire_compact_body<1024>(maxit_all, maxit, early_stop, alist, tmp, nact_p, unsat, mism, iters, status, rnd, done,
                            ndone, wsum, &base_s);
}

// Syndromes of the active frames and, in the workgroup that finishes last, the
// stopping rule and compaction (k_retire_compact's work), in one launch: every
// workgroup that checked a frame publishes its flags (device-scope release),
// every workgroup takes a ticket, and the holder of the last ticket acquires
// the flags and retires.  No workgroup waits for another.  A release writes
// back the XCD's L2, so this form is for passes with few active frames (a few
// releases); *ticket is zero on entry and reset by the last workgroup.
__global__ __launch_bounds__(256) void k_syndrome_retire(DevCode cd, const uint8_t* __restrict__ hard,
                                                         const uint8_t* __restrict__ fsw, uint8_t* __restrict__ synd,
                                                         uint32_t* unsat, uint32_t* mism, int* alist, int* nact_p,
                                                         int* rnd, int maxit_all, const int* __restrict__ maxit,
                                                         int early_stop, int* tmp, int32_t* iters,
                                                         uint32_t* status, int* done, int* ndone, unsigned* ticket) {
  extern __shared__ uint32_t smw[];
  __shared__ uint8_t s_exp[512];
  __shared__ uint16_t s_log[256];
  __shared__ int wsum[4];
  __shared__ int base_s;
  __shared__ int last;
  const int nact = *nact_p;
  syndrome_frames_body(cd, hard, fsw, synd, nullptr, unsat, mism, alist, nact, nullptr, rnd, smw, s_exp, s_log);
  // thread 0 wrote this workgroup's flags (after the body's last barrier)
  if (threadIdx.x == 0) {
    if ((int)blockIdx.x < nact) __threadfence();
    last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  retire_compact_body<256>(maxit_all, maxit, early_stop, alist, tmp, nact_p, unsat, mism, iters, status, rnd, done,
                           ndone, wsum, &base_s);
  if (threadIdx.x == 0) *ticket = 0u;
}

// Batched retirement after a run of R passes of the edge-parallel pass in its
// history form (k_fused_split HIST) over at most kHistSlots active frames, in
// place of a syndrome and retirement launch after every pass; two launches.
// k_tail_syndromes, one workgroup per (run pass r, slot): the frame's
// decision of round l = rnd[f] + r (rows hist_hard[r][slot],
// hist_fsw[r][slot]; none at round 0 or past the frame's last round) is
// checked as k_syndrome_retire checks it: direct syndrome row to
// hist_synd[r][slot], flags hist_flag[r][slot] (bit 0 some check nonzero,
// bit 1 the two syndromes differ).  k_tail_retire, one workgroup: the first
// round that stops each frame (both syndromes zero with early stopping, or
// its last round) gives its outputs (hard and synd from that round, iters = l,
// status with the mismatch bits of the rounds up to it and the converged
// bit); a frame that does not stop has iters set to its last round and rnd
// advanced by R; the active list is compacted in order (stopped frames
// appended to `done`).  The rounds the run made after a frame's stopping round
// only overwrote its message state (which the decode-time posterior calls then
// refuse to read).
constexpr int kHistRounds = 32, kHistSlots = 128;

__global__ __launch_bounds__(256) void k_tail_syndromes(DevCode cd, int S, const uint8_t* __restrict__ hist_hard,
                                                        const uint8_t* __restrict__ hist_fsw,
                                                        uint8_t* __restrict__ hist_synd, uint32_t* __restrict__ hist_flag,
                                                        const int* __restrict__ alist, const int* __restrict__ nact_p,
                                                        const int* __restrict__ rnd, int maxit_all,
                                                        const int* __restrict__ maxit) {
  extern __shared__ uint32_t smw[];   // [N] decisions, [E] sign words (bytes, word-rounded)
  __shared__ uint8_t s_exp[512];
  __shared__ uint16_t s_log[256];
  __shared__ int red[2];
  const int tid = threadIdx.x;
  const int r = blockIdx.x / S, slot = blockIdx.x % S;
  const int nact = *nact_p;
  if (slot >= nact) return;            // uniform over the block
  const int f = alist[slot];
  const int ell = rnd[f] + r;
  const int mi = maxit ? maxit[f] : maxit_all;
  if (ell < 1 || ell > mi) return;
  const int nw = (cd.N + 3) >> 2;
  uint8_t* sh = reinterpret_cast<uint8_t*>(smw);
  uint8_t* sw = reinterpret_cast<uint8_t*>(smw + nw);
  const uint8_t* hh = hist_hard + ((size_t)r * kHistSlots + slot) * cd.N;
  const uint8_t* hf = hist_fsw + ((size_t)r * kHistSlots + slot) * cd.E;
  for (int i = tid; i < 512; i += blockDim.x) s_exp[i] = cd.gexp[i];
  for (int i = tid; i < 256; i += blockDim.x) s_log[i] = cd.glog[i];
  for (int i = tid; i < cd.N; i += blockDim.x) sh[i] = hh[i];
  for (int i = tid; i < cd.E; i += blockDim.x) sw[i] = hf[i];
  if (tid == 0) {
    red[0] = 0;
    red[1] = 0;
  }
  __syncthreads();
  uint8_t* sy = hist_synd + ((size_t)r * kHistSlots + slot) * cd.M;
  int bad = 0, mm = 0;
  for (int c = tid; c < cd.M; c += blockDim.x) {
    const int e0 = cd.row_ptr[c], e1 = cd.row_ptr[c + 1];
    int sd = 0, sf = 0;
    for (int e = e0; e < e1; ++e) {
      const uint32_t pk = cd.e_pack[e];
      const int x = sh[pk & 0xFFFFFFu];
      if (x) sd ^= s_exp[s_log[pk >> 24] + s_log[x]];
      sf ^= sw[e];
    }
    sy[c] = (uint8_t)sd;
    bad |= sd | sf;
    mm |= sd != sf;
  }
  if (bad) atomicOr(&red[0], 1);
  if (mm) atomicOr(&red[1], 1);
  __syncthreads();
  if (tid == 0) hist_flag[(size_t)r * kHistSlots + slot] = (red[0] ? 1u : 0u) | (red[1] ? 2u : 0u);
}

__global__ __launch_bounds__(256) void k_tail_retire(DevCode cd, int R, const uint8_t* __restrict__ hist_hard,
                                                     const uint8_t* __restrict__ hist_synd,
                                                     const uint32_t* __restrict__ hist_flag,
                                                     uint8_t* __restrict__ hard, uint8_t* __restrict__ synd,
                                                     int* alist, int* nact_p, int* rnd, int maxit_all,
                                                     const int* __restrict__ maxit, int early_stop,
                                                     int32_t* iters, uint32_t* status, int* done, int* ndone) {
  __shared__ uint32_t s_flag[kHistRounds * kHistSlots];
  __shared__ int stop_r[kHistSlots];   // stopping run pass of each slot, -1: continues
  __shared__ int wsum[4];
  const int tid = threadIdx.x;
  const int nact = *nact_p;            // at most kHistSlots
  // the run's flags to LDS, four independent loads in flight per thread
  // (entries of rounds a frame did not check are read but never used)
  const int nf = R * kHistSlots;
  for (int i0 = 0; i0 < nf; i0 += 4 * 256) {
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 256 + tid;
      v[u] = i < nf ? hist_flag[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 256 + tid;
      if (i < nf) s_flag[i] = v[u];
    }
  }
  __syncthreads();
  if (tid < nact) {
    const int slot = tid;
    const int f = alist[slot];
    const int r0 = rnd[f];
    const int mi = maxit ? maxit[f] : maxit_all;
    uint32_t st = status[f];
    int stop = -1, last_ell = 0;
    for (int r = 0; r < R && stop < 0; ++r) {
      const int ell = r0 + r;
      if (ell == 0) continue;           // the frame's first pass: no decision
      if (ell > mi) break;
      const uint32_t fl = s_flag[r * kHistSlots + slot];
      const bool conv = (fl & 1u) == 0;
      if (fl & 2u) st |= 2u;
      last_ell = ell;
      if ((conv && early_stop) || ell >= mi) {
        stop = r;
        if (conv) st |= 1u;
      }
    }
    if (last_ell >= 1) iters[f] = last_ell;
    status[f] = st;
    if (stop < 0) rnd[f] = r0 + R;
    stop_r[slot] = stop;
  }
  __syncthreads();
  // outputs of the stopped frames from their stopping round, one wave per slot
  const int lane = tid & 63, w = tid >> 6;
  for (int slot = w; slot < nact; slot += 4) {
    const int r = stop_r[slot];        // uniform over the wave
    if (r < 0) continue;
    const int f = alist[slot];
    const uint8_t* hh = hist_hard + ((size_t)r * kHistSlots + slot) * cd.N;
    const uint8_t* sy = hist_synd + ((size_t)r * kHistSlots + slot) * cd.M;
#pragma unroll 4
    for (int i = lane; i < cd.N; i += 64) hard[(size_t)f * cd.N + i] = hh[i];
#pragma unroll 4
    for (int c = lane; c < cd.M; c += 64) synd[(size_t)f * cd.M + c] = sy[c];
  }
  // stable compaction of the active list (one pass: nact <= 256)
  const int keep = tid < nact ? (stop_r[tid] < 0 ? 1 : 0) : 0;
  const int f = tid < nact ? alist[tid] : -1;
  if (done && tid < nact && !keep) done[atomicAdd(ndone, 1)] = f;
  const uint64_t b = __builtin_amdgcn_ballot_w64(keep);
  const int pre = __builtin_popcountll(b & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[w] = __builtin_popcountll(b);
  __syncthreads();
  int off = 0;
  for (int k = 0; k < w; ++k) off += wsum[k];
  __syncthreads();                     // every thread has read alist[tid] before it is rewritten
  if (keep) alist[off + pre] = f;
  if (tid == 0) *nact_p = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Low-bit message storage, emulated in place on FP32 message arrays: every
// stored word is replaced by the nearest word of a b-bit format.
//   kind 0 (Log-Fourier words, sign | -log2|P|): the sign and a (b-1)-bit
//     unsigned magnitude on the grid {0, step, ..., (2^(b-1) - 1) step}
//     (round to nearest, saturating);
//   kind 1 (linear Fourier values P in [-1, 1]): b-bit two's complement
//     fixed point with step 2^-(b-1) (round to nearest, saturating at
//     +-(1 - 2^-(b-1)) and -1);
//   kind 2 (Log-SP log2 pmfs, <= 0): b-bit unsigned -k * step, k = 0 ..
//     2^b - 1 (round to nearest, saturating).
__global__ void k_quantise(float* __restrict__ w, size_t n, int kind, int bits, float step) {
  const float top = (float)((1 << (bits - 1)) - 1);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float x = w[i];
    if (kind == 0) {
      const float k = __builtin_fminf(__builtin_rintf(__builtin_fabsf(x) / step), top);
      w[i] = __builtin_copysignf(k * step, x);
    } else if (kind == 2) {
      const float k = __builtin_fminf(__builtin_rintf(-x / step), (float)((1 << bits) - 1));
      w[i] = -k * step;
    } else {
      const float sc = (float)(1 << (bits - 1));
      const float k = __builtin_fminf(__builtin_fmaxf(__builtin_rintf(x * sc), -sc), top);
      w[i] = k / sc;
    }
  }
}

}  // namespace ldpcfd
