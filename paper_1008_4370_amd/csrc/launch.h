// Launchers of the field-size templated kernels.  Each field size GF(2^m),
// m = 2..8, is compiled in a translation unit of its own (kernels_q.hip with
// LDPC_FD_LOGQ = m), which defines these templates for LOGQ = m; the host
// translation unit selects one at run time with by_m().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lfsp_kernels.h"

namespace ldpcfd {

// One pass of the fused decoder over the active frames alist[0..*nact) (see
// k_fused).  buf0/buf1 are message buffers of storage type `prec`
// (LDPC_FD_FP32/FP16/BF16).  split: the edge-parallel pass (k_fused_split).
struct FusedArgs {
  DevCode cd;
  int Fmax;             // frames the grid is sized for (bound on *nact)
  const float* prior;   // prior factors [F][N][m] or symbol priors [F][N][q]
  void* buf0;
  void* buf1;
  uint8_t* hard;
  uint8_t* fsw;
  const int* alist;
  const int* nact;
  const int* rnd;
  const int* maxit;     // per-frame max_iter or NULL (then maxit_all)
  int maxit_all;
  int cap;              // grid cap of the full pass (workgroups)
  int ar;               // variable-node arithmetic form (kFp32, kFp64, kSymbolPrior, kProbPrior)
  bool mfma;            // decision transforms on the matrix cores
  int prec;             // storage type of the message buffers
  bool split;           // edge-parallel pass
  // edge-parallel pass in a batched retirement (k_fused_split HIST): pass
  // roff of the run, decisions to the rows hist_hard[slot][N], hist_fsw[slot][E]
  int roff = 0;
  uint8_t* hist_hard = nullptr;
  uint8_t* hist_fsw = nullptr;
};

// PLAIN decoder kernels (k_var_plain / k_check_plain).
struct PlainArgs {
  DevCode cd;
  int F;
  const float* llr;
  const float* in;      // check-to-variable (variable kernel) / variable-to-check (check kernel)
  float* out;
  uint8_t* hard;
  uint8_t* fsw;
  const uint32_t* active;
  int first;
};

// Wavefront-per-node kernels (Log-SP, general variable node, linear Fourier SP
// check node) over nf frames alist[0..nf) (0..nf-1 when alist is NULL).
struct NodeArgs {
  DevCode cd;
  int nf;
  const int* alist;
  int kmax, jmax;
  const float* llr;
  const float* in;
  float* out;
  uint8_t* hard;
  uint8_t* fsw;
  int first;
  bool lin;             // linear Fourier SP variable node (k_var_gen)
  bool log8 = false;    // LOGSP: in/out hold 8-bit log2-probability codes (LDPC_FD_LOG8)
};

// Each returns false when no kernel variant exists for (kmax, logr).
template <int LOGQ> bool fused_pass(int kmax, int logr, const FusedArgs& a, hipStream_t s);
template <int LOGQ> bool var_plain(int kmax, int logr, const PlainArgs& a, hipStream_t s);
template <int LOGQ> bool check_plain(int kmax, int logr, const PlainArgs& a, hipStream_t s);
template <int LOGQ> bool logsp_check(const NodeArgs& a, hipStream_t s);
template <int LOGQ> bool logsp_var(const NodeArgs& a, hipStream_t s);
template <int LOGQ> bool var_gen(const NodeArgs& a, hipStream_t s);
template <int LOGQ> bool fsp_check(const NodeArgs& a, hipStream_t s);

// Run fn(std::integral_constant<int, m>) for m = 2..8; false for other m.
template <class Fn>
bool by_m(int m, Fn&& fn) {
  switch (m) {
    case 2: return fn(std::integral_constant<int, 2>{});
    case 3: return fn(std::integral_constant<int, 3>{});
    case 4: return fn(std::integral_constant<int, 4>{});
    case 5: return fn(std::integral_constant<int, 5>{});
    case 6: return fn(std::integral_constant<int, 6>{});
    case 7: return fn(std::integral_constant<int, 7>{});
    case 8: return fn(std::integral_constant<int, 8>{});
    default: return false;
  }
}

}  // namespace ldpcfd
