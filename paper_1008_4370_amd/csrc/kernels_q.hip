// Field-size templated kernels and their launchers for one field size
// GF(2^LDPC_FD_LOGQ); compiled once per m = 2..8 (see launch.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "launch.h"
#include "ldpc_fd.h"
#include "lfsp_kernels.h"
#include "logsp_kernels.h"

#ifndef LDPC_FD_LOGQ
#error "LDPC_FD_LOGQ (log2 of the field size) must be defined"
#endif

namespace ldpcfd {
namespace {

// Kernel geometry of the Log-Fourier kernels: 2^LOGR entries per lane, rows
// of weight up to KMAX.
template <int LOGQ, int LOGR, int KMAX>
struct Impl {
  using G = Geo<LOGQ, LOGR>;
  static constexpr int kWaves = 4;
  static size_t lds() { return (size_t)kWaves * G::T * G::QP * sizeof(float); }
  static unsigned blocks(long items) { return (unsigned)((items + kWaves - 1) / kWaves); }

  static bool var_plain(const PlainArgs& a, hipStream_t s) {
    const long items = (long)((a.F + G::T - 1) / G::T) * a.cd.N;
    if (items == 0) return true;
    hipLaunchKernelGGL(k_var_plain<G>, dim3(blocks(items)), dim3(64 * kWaves), lds(), s, a.cd, a.F, a.llr, a.in,
                       a.out, a.hard, a.fsw, a.active, a.first);
    return true;
  }
  static bool check_plain(const PlainArgs& a, hipStream_t s) {
    const long items = (long)((a.F + G::T - 1) / G::T) * a.cd.M;
    if (items == 0) return true;
    hipLaunchKernelGGL((k_check_plain<G, KMAX>), dim3(blocks(items)), dim3(64 * kWaves), lds(), s, a.cd, a.F, a.in,
                       a.out, a.active);
    return true;
  }
  // Grid of the grid-stride fused pass: enough workgroups for the largest
  // possible active list, capped, and a multiple of the XCD count.
  static unsigned fused_blocks(const DevCode& cd, int Fmax, int cap) {
    const long items = (long)((Fmax + G::T - 1) / G::T) * cd.M;
    long b = std::min<long>(blocks(items), cap);
    b = (b + kXcds - 1) / kXcds * kXcds;
    return (unsigned)std::max<long>(b, kXcds);
  }
  // Edge-parallel pass (k_fused_split) over at most Fmax active frames: one
  // workgroup of KMAX wavefronts per (frame group, check), grid-stride.
  // Built forms: every variable-node form with FP32 storage; the default
  // form (kProbPrior) only with 16-bit storage, whose words are message pmfs
  // (the entry points reject the other combinations).
  template <typename S>
  static void fused_split(const FusedArgs& a, hipStream_t s) {
    const long items = (long)((a.Fmax + G::T - 1) / G::T) * a.cd.M;
    const dim3 grid((unsigned)std::min<long>(items, 65536)), block(64 * KMAX);
    const size_t lds_bytes = (size_t)2 * KMAX * G::T * G::QP * sizeof(float);
    S* b0 = (S*)a.buf0;
    S* b1 = (S*)a.buf1;
#define LFD_SPLIT(AR)                                                                                           \
  do {                                                                                                         \
    if (a.hist_hard)                                                                                           \
      hipLaunchKernelGGL((k_fused_split<G, KMAX, S, AR, true>), grid, block, lds_bytes, s, a.cd, a.prior, b0,   \
                         b1, a.hard, a.fsw, a.alist, a.nact, a.rnd, a.maxit, a.maxit_all, a.roff, a.hist_hard,  \
                         a.hist_fsw);                                                                          \
    else                                                                                                       \
      hipLaunchKernelGGL((k_fused_split<G, KMAX, S, AR, false>), grid, block, lds_bytes, s, a.cd, a.prior, b0,  \
                         b1, a.hard, a.fsw, a.alist, a.nact, a.rnd, a.maxit, a.maxit_all, 0, nullptr, nullptr); \
  } while (0)
    if constexpr (kPmfWords<S>) {
      LFD_SPLIT(kProbPrior);   // 16-bit storage: the default variable node only
    } else {
      if (a.ar == kFp64) {
        LFD_SPLIT(kFp64);
        return;
      }
      if (a.ar == kProbPrior) {
        LFD_SPLIT(kProbPrior);
        return;
      }
      if (a.ar == kSymbolPrior) {
        LFD_SPLIT(kSymbolPrior);
        return;
      }
      LFD_SPLIT(kFp32);
    }
#undef LFD_SPLIT
  }
  template <typename S>
  static void fused(const FusedArgs& a, hipStream_t s) {
    const dim3 grid(fused_blocks(a.cd, a.Fmax, a.cap)), block(64 * kWaves);
    S* b0 = (S*)a.buf0;
    S* b1 = (S*)a.buf1;
#define LFD_FUSED(AR, DM)                                                                                          \
  hipLaunchKernelGGL((k_fused<G, KMAX, S, AR, DM>), grid, block, lds(), s, a.cd, a.prior, b0, b1, a.hard, a.fsw, \
                     a.alist, a.nact, a.rnd, a.maxit, a.maxit_all)
    if constexpr (kPmfWords<S>) {
      LFD_FUSED(kProbPrior, false);   // 16-bit storage: the default variable node only
    } else {
      if constexpr (kMfmaDecision<G>) {
        if (a.mfma && a.ar == kFp32) {
          LFD_FUSED(kFp32, true);
          return;
        }
      }
      if (a.ar == kFp64) {
        LFD_FUSED(kFp64, false);
        return;
      }
      if (a.ar == kProbPrior) {
        LFD_FUSED(kProbPrior, false);
        return;
      }
      if (a.ar == kSymbolPrior) {
        LFD_FUSED(kSymbolPrior, false);
        return;
      }
      LFD_FUSED(kFp32, false);
    }
#undef LFD_FUSED
  }
  static bool fused_pass(const FusedArgs& a, hipStream_t s) {
    if (a.Fmax == 0) return true;
    auto run = [&](auto tag) {
      using S = decltype(tag);
      if (a.split)
        fused_split<S>(a, s);
      else
        fused<S>(a, s);
    };
    if (a.prec == LDPC_FD_FP32)
      run(float{});
    else if (a.prec == LDPC_FD_FP16)
      run(_Float16{});
    else
      run(bf16_t{});
    return true;
  }
};

// Kernel variant: rows of weight <= 8 have variants with 4, 8 or 16 entries
// per lane (log2 R = 2, 3, 4; 16 entries for q >= 16); rows of weight 9..16
// use 4 or 8.
template <int LOGQ, class Fn>
bool dispatch_q(int kmax, int logr, Fn&& fn) {
  if (kmax <= 8) {
    if constexpr (LOGQ >= 4) {
      if (logr == 4) return fn(Impl<LOGQ, 4, 8>{});
    }
    if constexpr (LOGQ >= 3) {
      if (logr == 3) return fn(Impl<LOGQ, 3, 8>{});
    }
    return fn(Impl<LOGQ, 2, 8>{});
  }
  if (kmax <= 16) {
    if constexpr (LOGQ >= 3) {
      if (logr == 3) return fn(Impl<LOGQ, 3, 16>{});
    }
    return fn(Impl<LOGQ, 2, 16>{});
  }
  return false;
}

// Conventional log-domain SP kernels (LDPC_FD_MODE_LOGSP) and the general
// variable node: one wavefront per (frame, node), grid-stride over at most
// kLsBlocks workgroups.
constexpr long kLsBlocks = 16384;
unsigned ls_grid(long items) { return (unsigned)std::max<long>(1, std::min(items, kLsBlocks)); }

}  // namespace

template <int LOGQ>
bool fused_pass(int kmax, int logr, const FusedArgs& a, hipStream_t s) {
  return dispatch_q<LOGQ>(kmax, logr, [&](auto impl) { return decltype(impl)::fused_pass(a, s); });
}

template <int LOGQ>
bool var_plain(int kmax, int logr, const PlainArgs& a, hipStream_t s) {
  return dispatch_q<LOGQ>(kmax, logr, [&](auto impl) { return decltype(impl)::var_plain(a, s); });
}

template <int LOGQ>
bool check_plain(int kmax, int logr, const PlainArgs& a, hipStream_t s) {
  return dispatch_q<LOGQ>(kmax, logr, [&](auto impl) { return decltype(impl)::check_plain(a, s); });
}

template <int LOGQ>
bool logsp_check(const NodeArgs& a, hipStream_t s) {
  const long items = (long)a.nf * a.cd.M;
  if (items == 0) return true;
  const size_t lds = (size_t)(3 * a.kmax + 1) * (1 << LOGQ) * sizeof(float);
  if (a.log8)
    hipLaunchKernelGGL((k_logsp_check<LOGQ, uint8_t>), dim3(ls_grid(items)), dim3(64), lds, s, a.cd, a.nf, a.alist,
                       a.kmax, (const uint8_t*)a.in, (uint8_t*)a.out);
  else
    hipLaunchKernelGGL((k_logsp_check<LOGQ, float>), dim3(ls_grid(items)), dim3(64), lds, s, a.cd, a.nf, a.alist,
                       a.kmax, a.in, a.out);
  return true;
}

template <int LOGQ>
bool logsp_var(const NodeArgs& a, hipStream_t s) {
  const long items = (long)a.nf * a.cd.N;
  if (items == 0) return true;
  const size_t lds = (size_t)a.jmax * (1 << LOGQ) * sizeof(float);
  if (a.log8)
    hipLaunchKernelGGL((k_logsp_var<LOGQ, uint8_t>), dim3(ls_grid(items)), dim3(64), lds, s, a.cd, a.nf, a.alist,
                       a.llr, (const uint8_t*)a.in, (uint8_t*)a.out, a.hard, a.fsw, a.first);
  else
    hipLaunchKernelGGL((k_logsp_var<LOGQ, float>), dim3(ls_grid(items)), dim3(64), lds, s, a.cd, a.nf, a.alist,
                       a.llr, a.in, a.out, a.hard, a.fsw, a.first);
  return true;
}

// Log-Fourier (lin = false) or linear Fourier (lin = true) variable node for
// any column weight.
template <int LOGQ>
bool var_gen(const NodeArgs& a, hipStream_t s) {
  const long items = (long)a.nf * a.cd.N;
  if (items == 0) return true;
  const size_t lds = (size_t)a.jmax * (1 << LOGQ) * sizeof(float);
  if (a.lin)
    hipLaunchKernelGGL((k_var_gen<LOGQ, true>), dim3(ls_grid(items)), dim3(64), lds, s, a.cd, a.nf, a.alist, a.llr,
                       a.in, a.out, a.hard, a.fsw, a.first);
  else
    hipLaunchKernelGGL((k_var_gen<LOGQ, false>), dim3(ls_grid(items)), dim3(64), lds, s, a.cd, a.nf, a.alist, a.llr,
                       a.in, a.out, a.hard, a.fsw, a.first);
  return true;
}

// Linear Fourier SP check node (LDPC_FD_MODE_FSP).
template <int LOGQ>
bool fsp_check(const NodeArgs& a, hipStream_t s) {
  const long items = (long)a.nf * a.cd.M;
  if (items == 0) return true;
  const size_t lds = (size_t)2 * a.kmax * (1 << LOGQ) * sizeof(float);
  hipLaunchKernelGGL(k_fsp_check<LOGQ>, dim3(ls_grid(items)), dim3(64), lds, s, a.cd, a.nf, a.alist, a.kmax, a.in,
                     a.out);
  return true;
}

template bool fused_pass<LDPC_FD_LOGQ>(int, int, const FusedArgs&, hipStream_t);
template bool var_plain<LDPC_FD_LOGQ>(int, int, const PlainArgs&, hipStream_t);
template bool check_plain<LDPC_FD_LOGQ>(int, int, const PlainArgs&, hipStream_t);
template bool logsp_check<LDPC_FD_LOGQ>(const NodeArgs&, hipStream_t);
template bool logsp_var<LDPC_FD_LOGQ>(const NodeArgs&, hipStream_t);
template bool var_gen<LDPC_FD_LOGQ>(const NodeArgs&, hipStream_t);
template bool fsp_check<LDPC_FD_LOGQ>(const NodeArgs&, hipStream_t);

}  // namespace ldpcfd
