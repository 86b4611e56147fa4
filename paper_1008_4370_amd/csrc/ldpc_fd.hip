// libldpcfd: C-ABI Log-Fourier SP decoder for (2,k) non-binary LDPC codes on
// gfx950.  Entry points are declared and documented in include/ldpc_fd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <type_traits>

#include "ldpc_fd.h"
#include "frame_kernels.h"
#include "launch.h"

using namespace ldpcfd;

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(LDPC_FD_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

const uint32_t kDefaultPoly[9] = {0, 0x3, 0x7, 0xB, 0x13, 0x25, 0x43, 0x89, 0x11D};

const char* const kPmfOnlyDefault =
    "16-bit storage holds message pmfs, which only the default variable node (PRECISE = 2) reads";

}  // namespace

struct ldpc_fd_code_s {
  int M = 0, N = 0, m = 0, q = 0, E = 0, kmax = 0;
  // largest column weight; regular: every column has weight 2 (the (2,k)
  // codes the fused decoder, the pool and the decode-time posteriors serve)
  int jmax = 0;
  bool regular = true;
  uint32_t poly = 0;
  // tuning (ldpc_fd_set_tuning): log2 entries per lane, fused grid cap, rounds per
  // host check, replay of captured round chunks
  int logr = 4, blocks = 2048, chunk = 4, graphs = 1;
  // chunks that start with at most tail_frames active frames use the variant
  // with 2^tail_logr entries per lane (shorter per-item latency)
  int tail_logr = 2, tail_frames = 128;
  // passes per captured chunk once a chunk starts in the tail form (0: chunk)
  int tail_chunk = 0;
  // passes in a decode's first captured chunk (0: chunk)
  int first_chunk = 0;
  // 1: tail chunks of at most kHistRounds passes over at most kHistSlots
  // frames retire once per chunk (k_tail_retire) instead of after every pass
  int batch_retire = 0;
  // workspaces whose last FUSED decode retired in batches: a frame that
  // stopped inside a batched chunk has its messages overwritten by the
  // chunk's later passes, so the decode-time posterior calls refuse them
  std::vector<const void*> batched_ws;
  bool workspace_batched(const void* ws) {
    std::lock_guard<std::mutex> lock(gmu);
    return std::find(batched_ws.begin(), batched_ws.end(), ws) != batched_ws.end();
  }
  // 1: such chunks run the edge-parallel pass (k_fused_split)
  int split = 1;
  // variable-node form of the fused pass (tuning key PRECISE): 0 = FP32 prior
  // butterflies, 1 = FP64 (see conv_prior_d), 2 = FP32 through the
  // convolution theorem with the channel pmf (conv_symbol_prior, prob_prior)
  int precise = 2;
  // 1: the tentative decision's transforms on the matrix cores (FP16 MFMA,
  // variants with 16 frames per wavefront)
  int mfma = 0;
  // emulated low-bit message storage of the PLAIN and FSP decoders: bits (0 =
  // off) and the magnitude step of Log-Fourier words in units of 2^-12
  int qbits = 0, qstep = 256;
  int device = 0;
  std::vector<void*> allocs;
  DevCode dev{};
  // Captured chunks of rounds of the fused decoder, keyed by everything their
  // kernel arguments depend on.
  struct GraphKey {
    int F, prec, chunk, max_iter, logr, blocks, tail, rgrid, sf, ar, early, batch;
    const void *ws, *llr, *hard, *synd, *iters, *status;
    bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
  };
  struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    std::vector<hipEvent_t> ev;  // per-round fused-pass start/stop events (profiling)
  };
  std::vector<GraphEntry> gcache;
  hipStream_t cap_stream = nullptr;
  std::mutex gmu;  // guards gcache and cap_stream
  void drop_graphs() {
    for (auto& g : gcache) {
      (void)hipGraphExecDestroy(g.exec);
      for (auto e : g.ev) (void)hipEventDestroy(e);
    }
    gcache.clear();
  }
  ~ldpc_fd_code_s() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

template <typename T>
int32_t upload(ldpc_fd_code_s* c, const std::vector<T>& h, const T** out) {
  void* d = nullptr;
  const size_t bytes = std::max<size_t>(h.size() * sizeof(T), 16);
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return fail(LDPC_FD_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocs.push_back(d);
  if (!h.empty()) HIP_TRY(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<const T*>(d);
  return LDPC_FD_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Arithmetic form of the fused variable node for the PRECISE tuning value.
int var_form(int precise) { return precise == 1 ? kFp64 : precise == 2 ? kProbPrior : kFp32; }

size_t msg_bytes(int prec) { return prec == LDPC_FD_FP32 ? 4 : 2; }

// Field-size dispatch of the templated kernels (defined per field size in
// kernels_q.hip).
bool run_fused(const ldpc_fd_code_s* c, int logr, const FusedArgs& a, hipStream_t s) {
  return by_m(c->m, [&](auto M) { return fused_pass<decltype(M)::value>(c->kmax, logr, a, s); });
}
bool run_var_plain(const ldpc_fd_code_s* c, const PlainArgs& a, hipStream_t s) {
  return by_m(c->m, [&](auto M) { return var_plain<decltype(M)::value>(c->kmax, c->logr, a, s); });
}
bool run_check_plain(const ldpc_fd_code_s* c, const PlainArgs& a, hipStream_t s) {
  return by_m(c->m, [&](auto M) { return check_plain<decltype(M)::value>(c->kmax, c->logr, a, s); });
}
bool run_logsp_check(const ldpc_fd_code_s* c, const NodeArgs& a, hipStream_t s) {
  return by_m(c->m, [&](auto M) { return logsp_check<decltype(M)::value>(a, s); });
}
bool run_logsp_var(const ldpc_fd_code_s* c, const NodeArgs& a, hipStream_t s) {
  return by_m(c->m, [&](auto M) { return logsp_var<decltype(M)::value>(a, s); });
}
bool run_var_gen(const ldpc_fd_code_s* c, const NodeArgs& a, hipStream_t s) {
  return by_m(c->m, [&](auto M) { return var_gen<decltype(M)::value>(a, s); });
}
bool run_fsp_check(const ldpc_fd_code_s* c, const NodeArgs& a, hipStream_t s) {
  return by_m(c->m, [&](auto M) { return fsp_check<decltype(M)::value>(a, s); });
}
PlainArgs plain_args(const ldpc_fd_code_s* c, int F, const float* llr, const float* in, float* out, uint8_t* hard,
                     uint8_t* fsw, const uint32_t* active, int first) {
  return PlainArgs{c->dev, F, llr, in, out, hard, fsw, active, first};
}
NodeArgs node_args(const ldpc_fd_code_s* c, int nf, const int* alist, const float* llr, const float* in, float* out,
                   uint8_t* hard, uint8_t* fsw, int first, bool lin = false) {
  return NodeArgs{c->dev, nf, alist, c->kmax, c->jmax, llr, in, out, hard, fsw, first, lin};
}

// Workspace carving -------------------------------------------------------
struct PlainWs {
  float* v2c;
  float* c2v;
  uint8_t* fsw;
  uint32_t* active;
  uint32_t* unsat;
  uint32_t* mism;
  uint32_t* count;
  int* alist;  // LOGSP: frames still active after the last retirement
};
struct FusedWs {
  float* prior;  // [F][N][m] tanh(L/2)
  void* buf[2];
  uint8_t* fsw;
  int* alist;
  int* tmp;
  uint32_t* unsat;
  uint32_t* mism;
  int* nact;       // nact[0]: active frames; nact[2]: syndrome/retire ticket
  int* rnd;  // [F] per-frame round
  // batched retirement (k_tail_syndromes, k_tail_retire): decisions, sign
  // words and syndromes of a run's passes [kHistRounds][kHistSlots][N] /
  // [..][E] / [..][M] and their check flags [kHistRounds][kHistSlots]; NULL
  // when the code's rows make them too large
  uint8_t* hist_hard;
  uint8_t* hist_fsw;
  uint8_t* hist_synd;
  uint32_t* hist_flag;
};

// Bytes of the batched retirement's history buffers (0: not used for this
// code, whose rows would take more than 64 MiB of them).
size_t hist_bytes(const ldpc_fd_code_s* c) {
  const size_t b = (size_t)kHistRounds * kHistSlots * ((size_t)c->N + c->E + c->M + 4);
  return b <= ((size_t)64 << 20) ? b : 0;
}

// esize: bytes per message entry (4; 1 for the LOGSP decoder's 8-bit codes).
size_t plain_layout(const ldpc_fd_code_s* c, int F, char* base, PlainWs* w, int esize = 4) {
  const size_t msg = align256((size_t)F * c->E * c->q * esize);
  size_t off = 0;
  auto take = [&](size_t n) { char* p = base ? base + off : nullptr; off += align256(n); return p; };
  char* p0 = take(msg);
  char* p1 = take(msg);
  char* p2 = take((size_t)F * c->E);
  char* p3 = take((size_t)F * 4);
  char* p4 = take((size_t)F * 4);
  char* p5 = take((size_t)F * 4);
  char* p6 = take(4);
  char* p7 = take((size_t)F * 4);
  if (w)
    *w = PlainWs{(float*)p0, (float*)p1, (uint8_t*)p2, (uint32_t*)p3, (uint32_t*)p4, (uint32_t*)p5, (uint32_t*)p6,
                 (int*)p7};
  return off;
}

size_t fused_layout(const ldpc_fd_code_s* c, int F, int prec, char* base, FusedWs* w) {
  const size_t msg = align256((size_t)F * c->E * c->q * msg_bytes(prec));
  size_t off = 0;
  auto take = [&](size_t n) { char* p = base ? base + off : nullptr; off += align256(n); return p; };
  char* pt = take((size_t)F * c->N * c->m * 4);
  char* b0 = take(msg);
  char* b1 = take(msg);
  char* p2 = take((size_t)F * c->E);
  char* p3 = take((size_t)F * 4);
  char* p4 = take((size_t)F * 4);
  char* p5 = take((size_t)F * 4);
  char* p6 = take((size_t)F * 4);
  char* p7 = take(16);
  char* p8 = take((size_t)F * 4);
  const bool hist = hist_bytes(c) > 0;
  char* h1 = hist ? take((size_t)kHistRounds * kHistSlots * c->N) : nullptr;
  char* h2 = hist ? take((size_t)kHistRounds * kHistSlots * c->E) : nullptr;
  char* h3 = hist ? take((size_t)kHistRounds * kHistSlots * c->M) : nullptr;
  char* h4 = hist ? take(4 * (size_t)kHistRounds * kHistSlots) : nullptr;
  if (w)
    *w = FusedWs{(float*)pt, {b0, b1}, (uint8_t*)p2, (int*)p3, (int*)p4, (uint32_t*)p5, (uint32_t*)p6, (int*)p7, (int*)p8,
                 (uint8_t*)h1, (uint8_t*)h2, (uint8_t*)h3, (uint32_t*)h4};
  return off;
}

thread_local int* t_pinned = nullptr;

int32_t read_count(const void* dptr, hipStream_t s, int* out) {
  if (!t_pinned) HIP_TRY(hipHostMalloc((void**)&t_pinned, 64, hipHostMallocDefault));
  HIP_TRY(hipMemcpyAsync(t_pinned, dptr, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = *t_pinned;
  return LDPC_FD_OK;
}

unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// Emulated low-bit storage (tuning key QUANT_BITS) of F frames' messages:
// kind 0 for Log-Fourier words, 1 for linear Fourier values, 2 for Log-SP
// log2 pmfs.
void launch_quantise(const ldpc_fd_code_s* c, int F, float* msg, int kind, hipStream_t s) {
  if (!c->qbits) return;
  const size_t n = (size_t)F * c->E * c->q;
  if (n == 0) return;
  hipLaunchKernelGGL(k_quantise, dim3((unsigned)std::min<size_t>((n + 255) / 256, 16384)), dim3(256), 0, s, msg, n,
                     kind, c->qbits, (float)c->qstep / 4096.0f);
}

// Prior factors tanh(L/2) of every frame, symbol and bit.
void launch_prior(const ldpc_fd_code_s* c, int F, const float* llr, float* prior, hipStream_t s) {
  const size_t n = (size_t)F * c->N * c->m;
  hipLaunchKernelGGL(k_prior_factors, dim3((unsigned)std::min<size_t>((n + 255) / 256, 8192)), dim3(256), 0, s, llr,
                     prior, n, c->precise ? 1 : 0);
}

// Conversions between the FP32 signed-log message layout and 16-bit pmf
// words (ldpc_fd_round's import and export), one workgroup per (frame, edge)
// vector, FP64 transforms.
template <typename S>
void launch_lambda_to_pmf(const ldpc_fd_code_s* c, int F, const float* in, S* out, hipStream_t s) {
  const long nvec = (long)F * c->E;
  hipLaunchKernelGGL(k_lambda_to_pmf<S>, dim3((unsigned)std::min<long>(nvec, 65536)), dim3(std::max(c->q, 64)),
                     c->q * sizeof(double), s, in, out, nvec, c->q);
}
template <typename S>
void launch_pmf_to_lambda(const ldpc_fd_code_s* c, int F, const S* in, float* out, hipStream_t s) {
  const long nvec = (long)F * c->E;
  hipLaunchKernelGGL(k_pmf_to_lambda<S>, dim3((unsigned)std::min<long>(nvec, 65536)), dim3(std::max(c->q, 64)),
                     c->q * sizeof(double), s, in, out, nvec, c->q);
}

// Syndromes of the current decisions for the active frames (alist/nact, or all
// F frames gated by `active`).
void launch_syndrome(const ldpc_fd_code_s* c, int F, const uint8_t* hard, const uint8_t* fsw, uint8_t* synd,
                     uint8_t* fsynd, uint32_t* unsat, uint32_t* mism, const int* alist, const int* nact,
                     const uint32_t* active, hipStream_t s, const int* rnd = nullptr) {
  const size_t lds = 4 * (size_t)(((c->N + 3) >> 2) + ((c->E + 3) >> 2));
  if (lds <= 60000) {
    hipLaunchKernelGGL(k_syndrome_frames, dim3((unsigned)std::min(F, 4096)), dim3(256), lds, s, c->dev, hard, fsw,
                       synd, fsynd, unsat, mism, alist, nact, F, active, rnd);
  } else {
    hipLaunchKernelGGL(k_syndrome, dim3(cdiv((long)F * c->M, 256)), dim3(256), 0, s, c->dev, hard, fsw, synd,
                       fsynd, unsat, mism, alist, nact, F, active, rnd);
  }
}

// Largest active count for which a pass's syndromes and retirement run as one
// launch (k_syndrome_retire: each workgroup that checked a frame issues a
// device-scope release, cheap for a few frames, tens of microseconds for
// thousands); above it the syndrome kernel and k_retire_compact.
constexpr int kRetireOneLaunchMax = 128;

// Workgroups of the one-launch form for a code with F frame slots whose pass
// starts with `left` active frames in the tail form, or 0 for the two-launch
// form.
// Frames the edge-parallel pass's grid covers for a chunk that starts with
// `left` active frames (at most the tail threshold): 32 or 128 when the
// count is within them, so that a high threshold does not size the grid of
// the last passes, which run over a few frames.  The active count only falls
// within a chunk, so the grid covers every active slot.
int split_frames(const ldpc_fd_code_s* c, int F, int left) {
  int cap = std::max(c->tail_frames, 1);
  if (left <= 32)
    cap = std::min(cap, 32);
  else if (left <= 128)
    cap = std::min(cap, 128);
  return std::max(1, std::min(F, cap));
}

int retire_grid(const ldpc_fd_code_s* c, int F, bool tail, int left) {
  if (!tail || left > kRetireOneLaunchMax) return 0;
  return std::min(split_frames(c, F, left), kRetireOneLaunchMax);
}

// Syndromes of the active frames, stopping rule and compaction.  tail_grid > 0
// (at most that many frames are active): one launch of k_syndrome_retire with
// tail_grid workgroups; otherwise the syndrome kernel and k_retire_compact.
// ticket = nact + 2 (zero between launches).
void launch_syndrome_retire(const ldpc_fd_code_s* c, int F, const uint8_t* hard, const uint8_t* fsw, uint8_t* synd,
                            uint32_t* unsat, uint32_t* mism, int* alist, int* nact, int* rnd, int maxit_all,
                            const int* maxit, int* tmp, int32_t* iters, uint32_t* status, int* done, int* ndone,
                            int tail_grid, hipStream_t s, int early_stop = 1) {
  const size_t lds = 4 * (size_t)(((c->N + 3) >> 2) + ((c->E + 3) >> 2));
  if (tail_grid > 0 && lds <= 60000) {
    hipLaunchKernelGGL(k_syndrome_retire, dim3((unsigned)std::min(F, tail_grid)), dim3(256), lds, s, c->dev, hard, fsw,
                       synd, unsat, mism, alist, nact, rnd, maxit_all, maxit, early_stop, tmp, iters, status, done,
                       ndone, (unsigned*)(nact + 2));
  } else {
    launch_syndrome(c, F, hard, fsw, synd, nullptr, unsat, mism, alist, nact, nullptr, s, rnd);
    hipLaunchKernelGGL(k_retire_compact, dim3(1), dim3(1024), 0, s, maxit_all, maxit, early_stop, alist, tmp, nact,
                       unsat, mism, iters, status, rnd, done, ndone);
  }
}

// Per-thread kernel timing (ldpc_fd_profile_*).
struct Profile {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
};
thread_local Profile t_prof;

// Run `launch` on stream s, bracketed by events when profiling is on.
template <class Fn>
void timed(int kernel, hipStream_t s, Fn&& launch) {
  if (!t_prof.on) {
    launch();
    return;
  }
  hipEvent_t a = t_prof.get(), b = t_prof.get();
  if (a) (void)hipEventRecord(a, s);
  launch();
  if (b) (void)hipEventRecord(b, s);
  if (a && b) t_prof.ev[kernel].emplace_back(a, b);
}

}  // namespace

// ===========================================================================
extern "C" {

const char* ldpc_fd_last_error(void) { return g_err.c_str(); }

int32_t ldpc_fd_create_code(int32_t M, int32_t N, int32_t m, const int32_t* row_ptr, const int32_t* col,
                            const uint16_t* val, uint32_t prim_poly, ldpc_fd_code* out) {
  if (!out) return fail(LDPC_FD_E_INVALID, "out is NULL");
  *out = nullptr;
  if (m < 2 || m > 8) return fail(LDPC_FD_E_UNSUPPORTED, "m must be in 2..8");
  if (M < 1 || N < 1 || !row_ptr || !col || !val) return fail(LDPC_FD_E_INVALID, "bad shape or NULL array");
  if (N >= (1 << 24)) return fail(LDPC_FD_E_UNSUPPORTED, "N must be below 2^24");
  const int q = 1 << m;
  if (row_ptr[0] != 0) return fail(LDPC_FD_E_INVALID, "row_ptr[0] != 0");
  for (int c = 0; c < M; ++c)
    if (row_ptr[c + 1] < row_ptr[c]) return fail(LDPC_FD_E_INVALID, "row_ptr not nondecreasing");
  const int E = row_ptr[M];
  if (E != 2 * N) {
    // column weights are checked below; E = 2N is implied by weight 2
  }
  std::vector<int> colw(N, 0);
  int kmax = 0;
  for (int c = 0; c < M; ++c) {
    const int d = row_ptr[c + 1] - row_ptr[c];
    if (d < 2) return fail(LDPC_FD_E_INVALID, "row " + std::to_string(c) + " has weight < 2");
    kmax = std::max(kmax, d);
    for (int e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
      if (col[e] < 0 || col[e] >= N) return fail(LDPC_FD_E_INVALID, "column index out of range");
      if (val[e] == 0 || val[e] >= q) return fail(LDPC_FD_E_INVALID, "label outside 1..2^m-1");
      for (int e2 = row_ptr[c]; e2 < e; ++e2)
        if (col[e2] == col[e]) return fail(LDPC_FD_E_INVALID, "duplicate entry (c,v)");
      colw[col[e]]++;
    }
  }
  int jmax = 0;
  bool regular = true;
  for (int v = 0; v < N; ++v) {
    if (colw[v] < 1) return fail(LDPC_FD_E_INVALID, "column " + std::to_string(v) + " has weight 0");
    jmax = std::max(jmax, colw[v]);
    regular = regular && colw[v] == 2;
  }
  if (kmax > 16) return fail(LDPC_FD_E_UNSUPPORTED, "row weight above 16");
  if (jmax > 16) return fail(LDPC_FD_E_UNSUPPORTED, "column weight above 16");
  const uint32_t poly = prim_poly ? prim_poly : kDefaultPoly[m];
  if ((poly >> m) != 1u) return fail(LDPC_FD_E_INVALID, "prim_poly must have degree m");
  // field tables from the primitive polynomial (alpha = x)
  std::vector<uint8_t> gexp(512, 0);
  std::vector<uint16_t> glog(256, 0);
  {
    uint32_t x = 1;
    for (int i = 0; i < q - 1; ++i) {
      if (i > 0 && x == 1) return fail(LDPC_FD_E_INVALID, "prim_poly is not primitive");
      gexp[i] = (uint8_t)x;
      glog[x] = (uint16_t)i;
      x <<= 1;
      if (x & (uint32_t)q) x ^= poly;
    }
    if (x != 1) return fail(LDPC_FD_E_INVALID, "prim_poly is not primitive");
    for (int i = q - 1; i < 512; ++i) gexp[i] = gexp[i % (q - 1)];
  }
  auto gmul = [&](int a, int b) -> int { return (a && b) ? gexp[(glog[a] + glog[b]) % (q - 1)] : 0; };
  std::vector<uint8_t> ginv(256, 0);
  std::vector<uint64_t> colsT(256, 0);
  for (int h = 1; h < q; ++h) {
    ginv[h] = (uint8_t)gexp[(q - 1 - glog[h]) % (q - 1)];
    uint64_t w = 0;
    for (int b = 0; b < m; ++b) {  // M_h^T e_b = row b of M_h, column j = bits of h*alpha^j
      int rowb = 0;
      for (int j = 0; j < m; ++j) rowb |= ((gmul(h, 1 << j) >> b) & 1) << j;
      w |= (uint64_t)rowb << (8 * b);
    }
    colsT[h] = w;
  }
  // graph tables
  std::vector<int> rp(row_ptr, row_ptr + M + 1), ev(col, col + E), eo(E, -1), ve(2 * N, -1);
  std::vector<uint8_t> el(E);
  std::vector<uint32_t> epk(E);
  for (int e = 0; e < E; ++e) {
    el[e] = (uint8_t)val[e];
    epk[e] = (uint32_t)col[e] | ((uint32_t)val[e] << 24);
  }
  // edges of each variable in ascending order: CSR (v_ptr, v_list) for every
  // code, and the [N][2] table plus the other-edge map for regular ones
  std::vector<int> vp(N + 1, 0), vl(E);
  for (int v = 0; v < N; ++v) vp[v + 1] = vp[v] + colw[v];
  {
    std::vector<int> fill(N, 0);
    for (int e = 0; e < E; ++e) vl[vp[col[e]] + fill[col[e]]++] = e;
  }
  if (regular) {
    for (int v = 0; v < N; ++v) {
      ve[2 * v] = vl[vp[v]];
      ve[2 * v + 1] = vl[vp[v] + 1];
      eo[ve[2 * v]] = ve[2 * v + 1];
      eo[ve[2 * v + 1]] = ve[2 * v];
    }
  }
  auto* c = new (std::nothrow) ldpc_fd_code_s();
  if (!c) return fail(LDPC_FD_E_NOMEM, "host allocation failed");
  c->M = M; c->N = N; c->m = m; c->q = q; c->E = E; c->kmax = kmax; c->poly = poly;
  c->jmax = jmax; c->regular = regular;
  c->logr = kmax > 8 ? 2 : m <= 3 ? m : m <= 7 ? 4 : 3;
  (void)hipGetDevice(&c->device);
  DevCode& d = c->dev;
  d.M = M; d.N = N; d.E = E; d.m = m;
  int32_t rc;
  if ((rc = upload(c, rp, &d.row_ptr)) || (rc = upload(c, ev, &d.e_var)) || (rc = upload(c, eo, &d.e_other)) ||
      (rc = upload(c, el, &d.e_label)) || (rc = upload(c, ve, &d.v_edges)) || (rc = upload(c, colsT, &d.colsT)) ||
      (rc = upload(c, ginv, &d.ginv)) || (rc = upload(c, gexp, &d.gexp)) || (rc = upload(c, glog, &d.glog)) ||
      (rc = upload(c, epk, &d.e_pack)) || (rc = upload(c, vp, &d.v_ptr)) || (rc = upload(c, vl, &d.v_list))) {
    delete c;
    return rc;
  }
  *out = c;
  return LDPC_FD_OK;
}

int32_t ldpc_fd_destroy_code(ldpc_fd_code code) {
  delete code;
  return LDPC_FD_OK;
}

int32_t ldpc_fd_code_info(ldpc_fd_code c, int32_t* M, int32_t* N, int32_t* m, int32_t* E, int32_t* kmax) {
  if (!c) return fail(LDPC_FD_E_INVALID, "code is NULL");
  if (M) *M = c->M;
  if (N) *N = c->N;
  if (m) *m = c->m;
  if (E) *E = c->E;
  if (kmax) *kmax = c->kmax;
  return LDPC_FD_OK;
}

int32_t ldpc_fd_workspace_bytes(ldpc_fd_code c, int32_t frames, int32_t prec, int32_t mode, int64_t* bytes) {
  if (!c || !bytes || frames < 0) return fail(LDPC_FD_E_INVALID, "bad argument");
  if (prec < 0 || prec > 3) return fail(LDPC_FD_E_INVALID, "unknown precision");
  if (prec == LDPC_FD_LOG8 && mode != LDPC_FD_MODE_LOGSP)
    return fail(LDPC_FD_E_UNSUPPORTED, "8-bit log2-probability storage is for the LOGSP decoder");
  if (mode == LDPC_FD_MODE_PLAIN || mode == LDPC_FD_MODE_LOGSP || mode == LDPC_FD_MODE_FSP) {
    if (prec != LDPC_FD_FP32 && prec != LDPC_FD_LOG8)
      return fail(LDPC_FD_E_UNSUPPORTED, "PLAIN, LOGSP and FSP decoders store FP32 messages (LOGSP also LOG8)");
    *bytes = (int64_t)plain_layout(c, frames, nullptr, nullptr, prec == LDPC_FD_LOG8 ? 1 : 4);
  } else if (mode == LDPC_FD_MODE_FUSED) {
    *bytes = (int64_t)fused_layout(c, frames, prec, nullptr, nullptr);
  } else {
    return fail(LDPC_FD_E_INVALID, "unknown mode");
  }
  return LDPC_FD_OK;
}

namespace {

// Decode from BPSK LLRs (llr) or from symbol priors (prior, FUSED mode only).
// flags: LDPC_FD_FLAG_NO_EARLY_STOP and LDPC_FD_FLAG_ASYNC (see ldpc_fd_decode_ex).
int32_t decode_impl(ldpc_fd_code c, int32_t F, const float* llr, const float* prior, int32_t max_iter, int32_t prec,
                    int32_t mode, uint8_t* hard, uint8_t* synd, int32_t* iters, uint32_t* status, void* workspace,
                    int64_t workspace_bytes, void* stream, uint32_t flags = 0) {
  if (!c) return fail(LDPC_FD_E_INVALID, "code is NULL");
  const int early = (flags & LDPC_FD_FLAG_NO_EARLY_STOP) ? 0 : 1;
  const bool async = (flags & LDPC_FD_FLAG_ASYNC) != 0;
  if (async && (mode == LDPC_FD_MODE_LOGSP || mode == LDPC_FD_MODE_FSP || (mode == LDPC_FD_MODE_PLAIN && !c->regular)))
    return fail(LDPC_FD_E_UNSUPPORTED, "asynchronous decoding: FUSED and regular PLAIN only (the list-based "
                                       "decoders size each round from the host)");
  if (F < 0 || max_iter < 1) return fail(LDPC_FD_E_INVALID, "frames < 0 or max_iter < 1");
  if (F == 0) return LDPC_FD_OK;
  if (!(llr || prior) || !hard || !synd || !iters || !status || !workspace)
    return fail(LDPC_FD_E_INVALID, "NULL buffer");
  if (prior && mode != LDPC_FD_MODE_FUSED) return fail(LDPC_FD_E_UNSUPPORTED, "symbol priors need the FUSED mode");
  if (mode == LDPC_FD_MODE_FUSED && !c->regular)
    return fail(LDPC_FD_E_UNSUPPORTED, "the FUSED decoder needs column weight 2 (PLAIN and LOGSP take any)");
  if (prior && prec != LDPC_FD_FP32) return fail(LDPC_FD_E_UNSUPPORTED, "symbol priors need FP32 storage");
  if (!prior && c->precise != 2 && prec != LDPC_FD_FP32 && mode == LDPC_FD_MODE_FUSED)
    return fail(LDPC_FD_E_UNSUPPORTED, kPmfOnlyDefault);
  int64_t need = 0;
  int32_t rc = ldpc_fd_workspace_bytes(c, F, prec, mode, &need);
  if (rc) return rc;
  if (workspace_bytes < need) return fail(LDPC_FD_E_NOMEM, "workspace too small: need " + std::to_string(need));
  hipStream_t s = (hipStream_t)stream;
  const DevCode& cd = c->dev;
  const unsigned fb = cdiv(F, 256);
  if (mode == LDPC_FD_MODE_LOGSP) {
    // Flooding rounds over the list of still-active frames: round 1 takes all
    // F frames in order; each retirement appends the continuing frames to
    // w.alist (in any order: frames are independent) and the host reads their
    // count, which sizes the next round's launches.
    // LOG8: the message arrays hold one byte per entry (the emulated
    // QUANT_BITS grid does not apply)
    const bool log8 = prec == LDPC_FD_LOG8;
    PlainWs w;
    plain_layout(c, F, (char*)workspace, &w, log8 ? 1 : 4);
    hipLaunchKernelGGL(k_init_frames, dim3(fb), dim3(256), 0, s, F, w.active, w.unsat, w.mism, (int*)nullptr,
                       (int*)nullptr, iters, status, (int*)nullptr, 0);
    auto args = [&](int nf, const int* list, const float* l, const float* in, float* out, uint8_t* hd, uint8_t* fw,
                    int first) {
      NodeArgs a = node_args(c, nf, list, l, in, out, hd, fw, first);
      a.log8 = log8;
      return a;
    };
    auto quant = [&](float* msg) {
      if (!log8) launch_quantise(c, F, msg, 2, s);
    };
    bool ok = true;
    timed(LDPC_FD_K_VAR, s, [&] { ok = run_logsp_var(c, args(F, nullptr, llr, nullptr, w.v2c, hard, w.fsw, 1), s); });
    if (!ok) return fail(LDPC_FD_E_UNSUPPORTED, "no kernel for this code");
    quant(w.v2c);
    int nf = F;
    const int* list = nullptr;
    for (int ell = 1; ell <= max_iter; ++ell) {
      timed(LDPC_FD_K_CHECK, s, [&] { run_logsp_check(c, args(nf, list, nullptr, w.v2c, w.c2v, nullptr, nullptr, 0), s); });
      quant(w.c2v);
      timed(LDPC_FD_K_VAR, s, [&] { run_logsp_var(c, args(nf, list, llr, w.c2v, w.v2c, hard, w.fsw, 0), s); });
      quant(w.v2c);
      launch_syndrome(c, F, hard, w.fsw, synd, nullptr, w.unsat, w.mism, nullptr, nullptr, w.active, s);
      HIP_TRY(hipMemsetAsync(w.count, 0, 4, s));
      hipLaunchKernelGGL(k_retire_plain, dim3(fb), dim3(256), 0, s, F, ell, max_iter, w.active, w.unsat, w.mism,
                         iters, status, w.count, w.alist, early);
      int left = 0;
      if ((rc = read_count(w.count, s, &left))) return rc;
      if (left == 0) break;
      nf = left;
      list = w.alist;
    }
    HIP_TRY(hipGetLastError());
    return LDPC_FD_OK;
  }
  if (mode == LDPC_FD_MODE_FSP || (mode == LDPC_FD_MODE_PLAIN && !c->regular)) {
    // The general variable node over the list of active frames (compacted as
    // in the LOGSP loop) with, for FSP, the linear check node over the same
    // list, and otherwise the PLAIN check kernel gated by the active flags
    // (column weights other than 2).
    const bool lin = mode == LDPC_FD_MODE_FSP;
    const int qk = lin ? 1 : 0;
    PlainWs w;
    plain_layout(c, F, (char*)workspace, &w);
    hipLaunchKernelGGL(k_init_frames, dim3(fb), dim3(256), 0, s, F, w.active, w.unsat, w.mism, (int*)nullptr,
                       (int*)nullptr, iters, status, (int*)nullptr, 0);
    bool ok = true;
    timed(LDPC_FD_K_VAR, s, [&] { ok = run_var_gen(c, node_args(c, F, nullptr, llr, nullptr, w.v2c, hard, w.fsw, 1, lin), s); });
    if (!ok) return fail(LDPC_FD_E_UNSUPPORTED, "no kernel for this code");
    launch_quantise(c, F, w.v2c, qk, s);
    int nf = F;
    const int* list = nullptr;
    for (int ell = 1; ell <= max_iter; ++ell) {
      if (lin)
        timed(LDPC_FD_K_CHECK, s, [&] { run_fsp_check(c, node_args(c, nf, list, nullptr, w.v2c, w.c2v, nullptr, nullptr, 0), s); });
      else
        timed(LDPC_FD_K_CHECK, s, [&] { run_check_plain(c, plain_args(c, F, nullptr, w.v2c, w.c2v, nullptr, nullptr, w.active, 0), s); });
      launch_quantise(c, F, w.c2v, qk, s);
      timed(LDPC_FD_K_VAR, s, [&] { run_var_gen(c, node_args(c, nf, list, llr, w.c2v, w.v2c, hard, w.fsw, 0, lin), s); });
      launch_quantise(c, F, w.v2c, qk, s);
      launch_syndrome(c, F, hard, w.fsw, synd, nullptr, w.unsat, w.mism, nullptr, nullptr, w.active, s);
      HIP_TRY(hipMemsetAsync(w.count, 0, 4, s));
      hipLaunchKernelGGL(k_retire_plain, dim3(fb), dim3(256), 0, s, F, ell, max_iter, w.active, w.unsat, w.mism,
                         iters, status, w.count, w.alist, early);
      int left = 0;
      if ((rc = read_count(w.count, s, &left))) return rc;
      if (left == 0) break;
      nf = left;
      list = w.alist;
    }
    HIP_TRY(hipGetLastError());
    return LDPC_FD_OK;
  }
  if (mode == LDPC_FD_MODE_PLAIN) {
    PlainWs w;
    plain_layout(c, F, (char*)workspace, &w);
    hipLaunchKernelGGL(k_init_frames, dim3(fb), dim3(256), 0, s, F, w.active, w.unsat, w.mism, (int*)nullptr,
                       (int*)nullptr, iters, status, (int*)nullptr, 0);
    bool ok = true;
    timed(LDPC_FD_K_VAR, s, [&] { ok = run_var_plain(c, plain_args(c, F, llr, nullptr, w.v2c, hard, w.fsw, w.active, 1), s); });
    launch_quantise(c, F, w.v2c, 0, s);
    if (!ok) return fail(LDPC_FD_E_UNSUPPORTED, "no kernel for this code");
    for (int ell = 1; ell <= max_iter; ++ell) {
      timed(LDPC_FD_K_CHECK, s, [&] { run_check_plain(c, plain_args(c, F, nullptr, w.v2c, w.c2v, nullptr, nullptr, w.active, 0), s); });
      launch_quantise(c, F, w.c2v, 0, s);
      timed(LDPC_FD_K_VAR, s, [&] { run_var_plain(c, plain_args(c, F, llr, w.c2v, w.v2c, hard, w.fsw, w.active, 0), s); });
      launch_quantise(c, F, w.v2c, 0, s);
      launch_syndrome(c, F, hard, w.fsw, synd, nullptr, w.unsat, w.mism, nullptr, nullptr, w.active, s);
      HIP_TRY(hipMemsetAsync(w.count, 0, 4, s));
      hipLaunchKernelGGL(k_retire_plain, dim3(fb), dim3(256), 0, s, F, ell, max_iter, w.active, w.unsat, w.mism,
                         iters, status, w.count, (int*)nullptr, early);
      if (async) continue;   // every round is enqueued; the kernels skip stopped frames
      int left = 0;
      if ((rc = read_count(w.count, s, &left))) return rc;
      if (left == 0) break;
    }
    HIP_TRY(hipGetLastError());
    return LDPC_FD_OK;
  }
  if (mode != LDPC_FD_MODE_FUSED) return fail(LDPC_FD_E_INVALID, "unknown mode");
  {
    // until a batched chunk runs, this workspace will hold stopping-round messages
    std::lock_guard<std::mutex> lock(c->gmu);
    auto& v = c->batched_ws;
    v.erase(std::remove(v.begin(), v.end(), (const void*)workspace), v.end());
  }
  FusedWs w;
  fused_layout(c, F, prec, (char*)workspace, &w);
  hipLaunchKernelGGL(k_init_frames, dim3(fb), dim3(256), 0, s, F, (uint32_t*)nullptr, w.unsat, w.mism, w.alist,
                     w.nact, iters, status, w.rnd, 0);
  // the variable node's channel input: prior factors formed from the LLRs, or
  // the caller's symbol priors read in place
  const float* tp = w.prior;
  if (prior)
    tp = prior;
  else
    launch_prior(c, F, llr, w.prior, s);
  const int ar = prior ? kSymbolPrior : var_form(c->precise);
  // One pass over the active frames (each at its own round, see k_fused),
  // syndromes of the decisions it formed, stopping rule and compaction.
  // sf: frames the edge-parallel pass covers (split_frames), used in the tail
  auto enqueue_round = [&](hipStream_t st, hipEvent_t e0, hipEvent_t e1, int lr, bool tail, int rgrid, int sf) {
    bool ok = true;
    if (e0) (void)hipEventRecord(e0, st);
    const bool split = tail && c->split;
    const FusedArgs fa{cd, split ? sf : F, tp, w.buf[0], w.buf[1], hard,
                       w.fsw, w.alist, w.nact, w.rnd, nullptr, max_iter, c->blocks, ar, c->mfma != 0, prec, split};
    ok = run_fused(c, lr, fa, st);
    if (e1) (void)hipEventRecord(e1, st);
    launch_syndrome_retire(c, F, hard, w.fsw, synd, w.unsat, w.mism, w.alist, w.nact, w.rnd, max_iter, nullptr, w.tmp,
                           iters, status, nullptr, nullptr, rgrid, st, early);
    return ok;
  };
  // Batched retirement: pass r of a run of edge-parallel passes writes its
  // decisions to the history rows of run pass r; after the run,
  // k_tail_syndromes checks every (pass, slot) and k_tail_retire retires.
  // tgrid: slots the run covers (split_frames of its starting count, at most kHistSlots)
  const size_t tlds = 4 * (size_t)(((c->N + 3) >> 2) + ((c->E + 3) >> 2));
  auto enqueue_hist = [&](hipStream_t st, int lr, int r, int tgrid) {
    FusedArgs fa{cd, tgrid, tp, w.buf[0], w.buf[1], hard, w.fsw, w.alist, w.nact, w.rnd, nullptr, max_iter,
                 c->blocks, ar, c->mfma != 0, prec, true};
    fa.roff = r;
    fa.hist_hard = w.hist_hard + (size_t)r * kHistSlots * c->N;
    fa.hist_fsw = w.hist_fsw + (size_t)r * kHistSlots * c->E;
    return run_fused(c, lr, fa, st);
  };
  auto enqueue_tail_retire = [&](hipStream_t st, int R, int tgrid) {
    hipLaunchKernelGGL(k_tail_syndromes, dim3((unsigned)(R * tgrid)), dim3(256), tlds, st, cd, tgrid, w.hist_hard,
                       w.hist_fsw, w.hist_synd, w.hist_flag, w.alist, w.nact, w.rnd, max_iter, (const int*)nullptr);
    hipLaunchKernelGGL(k_tail_retire, dim3(1), dim3(256), 0, st, cd, R, w.hist_hard, w.hist_synd, w.hist_flag, hard,
                       synd, w.alist, w.nact, w.rnd, max_iter, (const int*)nullptr, early, iters, status,
                       (int*)nullptr, (int*)nullptr);
  };
  // whether a chunk of ch passes that starts with `left` active frames retires once
  const bool val = (flags & LDPC_FD_FLAG_VALIDATION) != 0;   // the posterior follows: keep the messages
  auto batched = [&](bool tail, int left, int ch) {
    return !val && tail && c->split && c->batch_retire && w.hist_hard && left <= kHistSlots && ch <= kHistRounds &&
           tlds <= 60000;
  };
  // A frame needs at most max_iter + 1 passes (pass l forms round l's decision).
  const int passes = max_iter + 1;
  // Kernel timing needs per-launch events, which HIP cannot time inside a
  // replayed graph: profiled decodes launch every pass from the host.
  // Kernel variant of a chunk of passes, from the active count at its start.
  // (asynchronous decodes never learn the active count: full variant throughout)
  auto is_tail = [&](int left) { return !async && left <= c->tail_frames; };
  auto variant = [&](int left) { return is_tail(left) ? c->tail_logr : c->logr; };
  // passes in the first chunk (host read of the active count after them)
  const int first = c->first_chunk > 0 ? c->first_chunk : c->chunk;
  if (!c->graphs || t_prof.on) {
    int lr = variant(F);
    bool tail = is_tail(F);
    int rgrid = retire_grid(c, F, tail, F);
    int sf = split_frames(c, F, F);
    for (int p = 1, next = first; p <= passes; ++p) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (t_prof.on) {
        e0 = t_prof.get();
        e1 = t_prof.get();
        if (e0 && e1) t_prof.ev[LDPC_FD_K_FUSED].emplace_back(e0, e1);
      }
      if (!enqueue_round(s, e0, e1, lr, tail, rgrid, sf))
        return fail(LDPC_FD_E_UNSUPPORTED, "no kernel for this code");
      if (!async && (p == next || p == passes)) {
        int left = 0;
        if ((rc = read_count(w.nact, s, &left))) return rc;
        if (left == 0) break;
        lr = variant(left);
        tail = is_tail(left);
        rgrid = retire_grid(c, F, tail, left);
        sf = split_frames(c, F, left);
        next = p + c->chunk;
      }
    }
    HIP_TRY(hipGetLastError());
    return LDPC_FD_OK;
  }
  // Replay a captured chunk of passes; passes after every frame has stopped
  // find an empty active list and do nothing.
  const int chunk = c->chunk;
  std::lock_guard<std::mutex> lock(c->gmu);
  // The captured chunk for kernel variant lr (found in or added to the cache).
  auto chunk_graph = [&](int lr, bool tail, int rgrid, int sf, int chunk, bool batch, hipGraphExec_t* exec) -> int32_t {
    // zero-filled first: keys compare with memcmp, padding included
    ldpc_fd_code_s::GraphKey key;
    std::memset(&key, 0, sizeof key);
    key.F = F;
    key.prec = prec;
    key.chunk = chunk;
    key.max_iter = max_iter;
    key.logr = lr;
    key.blocks = c->blocks;
    key.tail = tail ? 1 : 0;
    key.rgrid = rgrid;
    key.sf = tail ? sf : 0;
    key.ar = ar;
    key.early = early;
    key.batch = batch ? 1 : 0;
    key.ws = workspace;
    key.llr = tp;
    key.hard = hard;
    key.synd = synd;
    key.iters = iters;
    key.status = status;
    for (auto& g : c->gcache)
      if (g.key == key) {
        *exec = g.exec;
        return LDPC_FD_OK;
      }
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (c->gcache.size() >= 8) c->drop_graphs();
    ldpc_fd_code_s::GraphEntry g{key, nullptr, {}};
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    bool ok = true;
    if (batch) {
      const int tgrid = std::min(sf, kHistSlots);
      for (int r = 0; r < chunk; ++r) ok = enqueue_hist(c->cap_stream, lr, r, tgrid) && ok;
      enqueue_tail_retire(c->cap_stream, chunk, tgrid);
    } else {
      for (int r = 0; r < chunk; ++r)
        ok = enqueue_round(c->cap_stream, nullptr, nullptr, lr, tail, rgrid, sf) && ok;
    }
    HIP_TRY(hipStreamEndCapture(c->cap_stream, &graph));
    if (!ok) {
      (void)hipGraphDestroy(graph);
      return fail(LDPC_FD_E_UNSUPPORTED, "no kernel for this code");
    }
    hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(LDPC_FD_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    c->gcache.push_back(g);
    *exec = g.exec;
    return LDPC_FD_OK;
  };
  int left = F;
  bool any_batch = false;
  // record whether this workspace's messages are those of the stopping rounds
  auto note_batch = [&]() {
    auto& v = c->batched_ws;
    if (any_batch && std::find(v.begin(), v.end(), (const void*)workspace) == v.end()) {
      if (v.size() >= 64) v.erase(v.begin());
      v.push_back(workspace);
    }
  };
  for (int p = 0, ch = chunk; p < passes; p += ch) {
    hipGraphExec_t exec = nullptr;
    const bool tail = is_tail(left);
    ch = tail && c->tail_chunk > 0 ? c->tail_chunk : p == 0 ? first : chunk;
    const bool batch = batched(tail, left, ch);
    any_batch = any_batch || batch;
    const int sf = split_frames(c, F, left);
    if ((rc = chunk_graph(variant(left), tail, batch ? 0 : retire_grid(c, F, tail, left), sf, ch, batch, &exec))) {
      note_batch();
      return rc;
    }
    HIP_TRY(hipGraphLaunch(exec, s));
    if (async) continue;   // passes after the last frame stops find no active frame
    if ((rc = read_count(w.nact, s, &left))) {
      note_batch();
      return rc;
    }
    if (left == 0) break;
  }
  note_batch();
  HIP_TRY(hipGetLastError());
  return LDPC_FD_OK;
}

}  // namespace

int32_t ldpc_fd_decode(ldpc_fd_code c, int32_t F, const float* llr, int32_t max_iter, int32_t prec, int32_t mode,
                       uint8_t* hard, uint8_t* synd, int32_t* iters, uint32_t* status, void* workspace,
                       int64_t workspace_bytes, void* stream) {
  if (F > 0 && !llr) return fail(LDPC_FD_E_INVALID, "NULL buffer");
  return decode_impl(c, F, llr, nullptr, max_iter, prec, mode, hard, synd, iters, status, workspace,
                     workspace_bytes, stream);
}

int32_t ldpc_fd_decode_prior(ldpc_fd_code c, int32_t F, const float* prior, int32_t max_iter, int32_t prec,
                             uint8_t* hard, uint8_t* synd, int32_t* iters, uint32_t* status, void* workspace,
                             int64_t workspace_bytes, void* stream) {
  if (F > 0 && !prior) return fail(LDPC_FD_E_INVALID, "NULL buffer");
  return decode_impl(c, F, nullptr, prior, max_iter, prec, LDPC_FD_MODE_FUSED, hard, synd, iters, status,
                     workspace, workspace_bytes, stream);
}

}  // extern "C"

// Device scratch of ldpc_fd_round_noalloc (see scratch_for_current_device).
constexpr size_t kRoundScratchBytes = (size_t)LDPC_FD_ROUND_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kRoundScratchBytes];

namespace {

// Argument checks of ldpc_fd_round and ldpc_fd_round_noalloc.
int32_t round_check(ldpc_fd_code c, int32_t F, const float* llr, const float* c2v_in, float* v2c_out,
                    float* c2v_out, uint8_t* hard, uint8_t* fsynd, uint8_t* synd, int32_t mode, int32_t prec) {
  if (!c) return fail(LDPC_FD_E_INVALID, "code is NULL");
  if (F < 0) return fail(LDPC_FD_E_INVALID, "frames < 0");
  if (F == 0) return LDPC_FD_OK;
  if (!llr || !c2v_out) return fail(LDPC_FD_E_INVALID, "NULL llr or c2v_out");
  if (c2v_in && (!hard || !fsynd || !synd)) return fail(LDPC_FD_E_INVALID, "decision outputs required");
  if (mode != LDPC_FD_MODE_FUSED && !v2c_out) return fail(LDPC_FD_E_INVALID, "PLAIN, LOGSP and FSP rounds need v2c_out");
  if (mode == LDPC_FD_MODE_FUSED && v2c_out) return fail(LDPC_FD_E_INVALID, "FUSED round does not form v2c_out");
  if (mode == LDPC_FD_MODE_FUSED && !c->regular)
    return fail(LDPC_FD_E_UNSUPPORTED, "the FUSED decoder needs column weight 2 (PLAIN and LOGSP take any)");
  if (mode == LDPC_FD_MODE_FUSED && c->precise != 2 && prec != LDPC_FD_FP32)
    return fail(LDPC_FD_E_UNSUPPORTED, kPmfOnlyDefault);
  if (mode < LDPC_FD_MODE_PLAIN || mode > LDPC_FD_MODE_FSP) return fail(LDPC_FD_E_INVALID, "unknown mode");
  if (prec == LDPC_FD_LOG8) return fail(LDPC_FD_E_UNSUPPORTED, "8-bit storage is for whole LOGSP decodes only");
  if (prec < 0 || prec > 2) return fail(LDPC_FD_E_INVALID, "unknown precision");
  if (mode != LDPC_FD_MODE_FUSED && prec != LDPC_FD_FP32)
    return fail(LDPC_FD_E_UNSUPPORTED, "PLAIN, LOGSP and FSP are FP32 only");
  return LDPC_FD_OK;
}

// Temporary device memory of one round (decision words, frame flags, 16-bit
// staging of the imported and exported state, prior factors, round counters).
struct RoundTmp {
  uint8_t* fsw;
  uint32_t *active, *unsat, *mism;
  int *alist, *nact, *rnd;
  char *st_in, *st_out;
  float* prior;
};

size_t round_layout(const ldpc_fd_code_s* c, int F, int prec, char* base, RoundTmp* t) {
  const size_t n_msg = (size_t)F * c->E * c->q;
  size_t off = 0;
  auto take = [&](size_t n) { char* p = base ? base + off : nullptr; off += align256(n); return p; };
  char* fsw = take((size_t)F * c->E);
  char* act = take((size_t)F * 4);
  char* uns = take((size_t)F * 4);
  char* mis = take((size_t)F * 4);
  char* al = take((size_t)F * 4);
  char* na = take(16);
  char* rn = take((size_t)F * 4);
  char* si = prec == LDPC_FD_FP32 ? nullptr : take(n_msg * 2);
  char* so = prec == LDPC_FD_FP32 ? nullptr : take(n_msg * 2);
  char* pr = take((size_t)F * c->N * c->m * 4);
  if (t)
    *t = RoundTmp{(uint8_t*)fsw, (uint32_t*)act, (uint32_t*)uns, (uint32_t*)mis, (int*)al, (int*)na, (int*)rn,
                  si, so, (float*)pr};
  return off;
}

// One flooding round (see ldpc_fd_round) with its temporaries carved from
// `tmp` (round_layout bytes); enqueued on `stream`, not synchronised.
int32_t round_impl(ldpc_fd_code c, int32_t F, const float* llr, const float* c2v_in, float* v2c_out, float* c2v_out,
                   uint8_t* hard, uint8_t* fsynd, uint8_t* synd, int32_t mode, int32_t prec, hipStream_t s,
                   char* tmp) {
  const DevCode& cd = c->dev;
  RoundTmp t;
  round_layout(c, F, prec, tmp, &t);
  const size_t n_msg = (size_t)F * c->E * c->q;
  uint8_t* fsw = t.fsw;
  uint32_t* active = t.active;
  uint32_t* unsat = t.unsat;
  uint32_t* mism = t.mism;
  int* alist = t.alist;
  int* nact = t.nact;
  int* rnd = t.rnd;
  float* prior = t.prior;
  const unsigned fb = cdiv(F, 256);
  hipLaunchKernelGGL(k_init_frames, dim3(fb), dim3(256), 0, s, F, active, unsat, mism, alist, nact, (int32_t*)nullptr,
                     (uint32_t*)nullptr, rnd, c2v_in ? 1 : 0);
  launch_prior(c, F, llr, prior, s);
  bool ok = true;
  const int first = c2v_in ? 0 : 1;
  if (mode == LDPC_FD_MODE_LOGSP) {
    ok = run_logsp_var(c, node_args(c, F, nullptr, llr, c2v_in, v2c_out, hard, fsw, first), s);
    launch_quantise(c, F, v2c_out, 2, s);
    if (c2v_in) launch_syndrome(c, F, hard, fsw, synd, fsynd, unsat, mism, nullptr, nullptr, nullptr, s);
    ok = ok && run_logsp_check(c, node_args(c, F, nullptr, nullptr, v2c_out, c2v_out, nullptr, nullptr, 0), s);
    launch_quantise(c, F, c2v_out, 2, s);
  } else if (mode == LDPC_FD_MODE_FSP || (mode == LDPC_FD_MODE_PLAIN && !c->regular)) {
    const bool lin = mode == LDPC_FD_MODE_FSP;
    ok = run_var_gen(c, node_args(c, F, nullptr, llr, c2v_in, v2c_out, hard, fsw, first, lin), s);
    launch_quantise(c, F, v2c_out, lin ? 1 : 0, s);
    if (c2v_in) launch_syndrome(c, F, hard, fsw, synd, fsynd, unsat, mism, nullptr, nullptr, nullptr, s);
    if (lin)
      ok = ok && run_fsp_check(c, node_args(c, F, nullptr, nullptr, v2c_out, c2v_out, nullptr, nullptr, 0), s);
    else
      ok = ok && run_check_plain(c, plain_args(c, F, nullptr, v2c_out, c2v_out, nullptr, nullptr, nullptr, 0), s);
    launch_quantise(c, F, c2v_out, lin ? 1 : 0, s);
  } else if (mode == LDPC_FD_MODE_PLAIN) {
    ok = run_var_plain(c, plain_args(c, F, llr, c2v_in, v2c_out, hard, fsw, nullptr, first), s);
    launch_quantise(c, F, v2c_out, 0, s);
    if (c2v_in) launch_syndrome(c, F, hard, fsw, synd, fsynd, unsat, mism, nullptr, nullptr, nullptr, s);
    ok = ok && run_check_plain(c, plain_args(c, F, nullptr, v2c_out, c2v_out, nullptr, nullptr, nullptr, 0), s);
    launch_quantise(c, F, c2v_out, 0, s);
  } else {
    // Frames at round 1 read buffer 1 and write buffer 0; frames at round 0
    // (no imported state) write buffer 1.  16-bit storage: the imported state
    // is converted to the stored word (the pmf times q, rounded) first and
    // the stored result converted back to normalised signed-log words.
    auto run = [&](auto tag) {
      using S = decltype(tag);
      S* in = (S*)c2v_in;
      S* out = (S*)c2v_out;
      if constexpr (kPmfWords<S>) {
        in = (S*)t.st_in;
        out = (S*)t.st_out;
        if (c2v_in) launch_lambda_to_pmf<S>(c, F, c2v_in, in, s);
      }
      const FusedArgs fa{cd, F, prior, c2v_in ? (void*)out : nullptr, c2v_in ? (void*)in : (void*)out, hard, fsw,
                         alist, nact, rnd, nullptr, 1 << 30, c->blocks, var_form(c->precise), c->mfma != 0, prec, false};
      ok = run_fused(c, c->logr, fa, s);
      if constexpr (kPmfWords<S>) launch_pmf_to_lambda<S>(c, F, (const S*)out, c2v_out, s);
    };
    if (prec == LDPC_FD_FP32) run(float{});
    else if (prec == LDPC_FD_FP16) run(_Float16{});
    else run(bf16_t{});
    if (c2v_in) launch_syndrome(c, F, hard, fsw, synd, fsynd, unsat, mism, alist, nact, nullptr, s, rnd);
  }
  if (!ok) return fail(LDPC_FD_E_UNSUPPORTED, "no kernel for this code");
  HIP_TRY(hipGetLastError());
  return LDPC_FD_OK;
}

// The scratch array exists once per GPU (each device holds its own copy at its
// own address until the process ends).  Host code never passes `scratch`
// itself to a kernel or a copy (in host code the name is a host-side
// stand-in); it uses the device address that hipGetSymbolAddress returns with
// the device current, looked up on the first call on each device and kept in
// g_scratch_ptr.

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_for_current_device(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LDPC_FD_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LDPC_FD_E_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return LDPC_FD_OK;
}

}  // namespace

extern "C" {

int32_t ldpc_fd_round(ldpc_fd_code c, int32_t F, const float* llr, const float* c2v_in, float* v2c_out,
                      float* c2v_out, uint8_t* hard, uint8_t* fsynd, uint8_t* synd, int32_t mode, int32_t prec,
                      void* stream) {
  int32_t rc = round_check(c, F, llr, c2v_in, v2c_out, c2v_out, hard, fsynd, synd, mode, prec);
  if (rc || F == 0) return rc;
  hipStream_t s = (hipStream_t)stream;
  char* tmp = nullptr;
  HIP_TRY(hipMalloc((void**)&tmp, round_layout(c, F, prec, nullptr, nullptr)));
  rc = round_impl(c, F, llr, c2v_in, v2c_out, c2v_out, hard, fsynd, synd, mode, prec, s, tmp);
  hipError_t e1 = hipStreamSynchronize(s);
  hipError_t e2 = hipFree(tmp);
  if (rc) return rc;
  if (e1 != hipSuccess) return fail(LDPC_FD_E_HIP, std::string("round: ") + hipGetErrorString(e1));
  if (e2 != hipSuccess) return fail(LDPC_FD_E_HIP, std::string("hipFree: ") + hipGetErrorString(e2));
  return LDPC_FD_OK;
}

int32_t ldpc_fd_round_noalloc(ldpc_fd_code c, int32_t F, const float* llr, const float* c2v_in, float* v2c_out,
                              float* c2v_out, uint8_t* hard, uint8_t* fsynd, uint8_t* synd, int32_t mode,
                              int32_t prec, void* stream) {
  int32_t rc = round_check(c, F, llr, c2v_in, v2c_out, c2v_out, hard, fsynd, synd, mode, prec);
  if (rc || F == 0) return rc;
  const size_t need = round_layout(c, F, prec, nullptr, nullptr);
  if (need > kRoundScratchBytes)
    return fail(LDPC_FD_E_NOMEM, "round needs " + std::to_string(need) + " bytes of scratch; the static array holds " +
                                     std::to_string(kRoundScratchBytes) + " (use fewer frames or ldpc_fd_round)");
  char* tmp = nullptr;
  if ((rc = scratch_for_current_device(&tmp))) return rc;
  return round_impl(c, F, llr, c2v_in, v2c_out, c2v_out, hard, fsynd, synd, mode, prec, (hipStream_t)stream, tmp);
}


int32_t ldpc_fd_set_tuning(ldpc_fd_code c, int32_t key, int32_t value) {
  if (!c) return fail(LDPC_FD_E_INVALID, "code is NULL");
  {
    std::lock_guard<std::mutex> lock(c->gmu);
    c->drop_graphs();
  }
  switch (key) {
    case LDPC_FD_TUNE_LANE_ENTRIES:
      if (value != 4 && value != 8 && value != 16) return fail(LDPC_FD_E_INVALID, "entries per lane: 4, 8 or 16");
      if (value > c->q || (value > 8 && c->kmax > 8))
        return fail(LDPC_FD_E_UNSUPPORTED, "no kernel variant with that many entries per lane for this code");
      c->logr = value == 4 ? 2 : value == 8 ? 3 : 4;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_GRID_BLOCKS:
      if (value < 8 || value > (1 << 20)) return fail(LDPC_FD_E_INVALID, "grid blocks outside 8..2^20");
      c->blocks = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_CHUNK:
      if (value < 1 || value > 1000) return fail(LDPC_FD_E_INVALID, "chunk outside 1..1000");
      c->chunk = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_GRAPHS:
      if (value != 0 && value != 1) return fail(LDPC_FD_E_INVALID, "graphs: 0 or 1");
      c->graphs = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_TAIL_ENTRIES:
      if (value != 4 && value != 8 && value != 16) return fail(LDPC_FD_E_INVALID, "entries per lane: 4, 8 or 16");
      if (value > c->q || (value > 8 && c->kmax > 8))
        return fail(LDPC_FD_E_UNSUPPORTED, "no kernel variant with that many entries per lane for this code");
      c->tail_logr = value == 4 ? 2 : value == 8 ? 3 : 4;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_TAIL_FRAMES:
      if (value < 0) return fail(LDPC_FD_E_INVALID, "tail frames < 0");
      c->tail_frames = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_PRECISE:
      if (value < 0 || value > 2) return fail(LDPC_FD_E_INVALID, "precise: 0, 1 or 2");
      c->precise = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_DECISION_MFMA:
      if (value != 0 && value != 1) return fail(LDPC_FD_E_INVALID, "decision MFMA: 0 or 1");
      c->mfma = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_TAIL_SPLIT:
      if (value != 0 && value != 1) return fail(LDPC_FD_E_INVALID, "tail split: 0 or 1");
      c->split = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_QUANT_BITS:
      if (value != 0 && (value < 3 || value > 16)) return fail(LDPC_FD_E_INVALID, "quantisation bits: 0 or 3..16");
      c->qbits = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_QUANT_STEP:
      if (value < 1 || value > (1 << 16)) return fail(LDPC_FD_E_INVALID, "quantisation step outside 1..65536");
      c->qstep = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_TAIL_CHUNK:
      if (value < 0 || value > 1000) return fail(LDPC_FD_E_INVALID, "tail chunk outside 0..1000");
      c->tail_chunk = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_BATCH_RETIRE:
      if (value != 0 && value != 1) return fail(LDPC_FD_E_INVALID, "batch retire: 0 or 1");
      c->batch_retire = value;
      return LDPC_FD_OK;
    case LDPC_FD_TUNE_FIRST_CHUNK:
      if (value < 0 || value > 1000) return fail(LDPC_FD_E_INVALID, "first chunk outside 0..1000");
      c->first_chunk = value;
      return LDPC_FD_OK;
    default:
      return fail(LDPC_FD_E_INVALID, "unknown tuning key");
  }
}

int32_t ldpc_fd_get_tuning(ldpc_fd_code c, int32_t key, int32_t* value) {
  if (!c || !value) return fail(LDPC_FD_E_INVALID, "NULL argument");
  switch (key) {
    case LDPC_FD_TUNE_LANE_ENTRIES: *value = 1 << c->logr; return LDPC_FD_OK;
    case LDPC_FD_TUNE_GRID_BLOCKS: *value = c->blocks; return LDPC_FD_OK;
    case LDPC_FD_TUNE_CHUNK: *value = c->chunk; return LDPC_FD_OK;
    case LDPC_FD_TUNE_GRAPHS: *value = c->graphs; return LDPC_FD_OK;
    case LDPC_FD_TUNE_TAIL_ENTRIES: *value = 1 << c->tail_logr; return LDPC_FD_OK;
    case LDPC_FD_TUNE_TAIL_FRAMES: *value = c->tail_frames; return LDPC_FD_OK;
    case LDPC_FD_TUNE_PRECISE: *value = c->precise; return LDPC_FD_OK;
    case LDPC_FD_TUNE_DECISION_MFMA: *value = c->mfma; return LDPC_FD_OK;
    case LDPC_FD_TUNE_TAIL_SPLIT: *value = c->split; return LDPC_FD_OK;
    case LDPC_FD_TUNE_QUANT_BITS: *value = c->qbits; return LDPC_FD_OK;
    case LDPC_FD_TUNE_QUANT_STEP: *value = c->qstep; return LDPC_FD_OK;
    case LDPC_FD_TUNE_TAIL_CHUNK: *value = c->tail_chunk; return LDPC_FD_OK;
    case LDPC_FD_TUNE_BATCH_RETIRE: *value = c->batch_retire; return LDPC_FD_OK;
    case LDPC_FD_TUNE_FIRST_CHUNK: *value = c->first_chunk; return LDPC_FD_OK;
    default: return fail(LDPC_FD_E_INVALID, "unknown tuning key");
  }
}

int32_t ldpc_fd_profile_enable(int32_t on) {
  t_prof.on = on != 0;
  return LDPC_FD_OK;
}

int32_t ldpc_fd_profile_read(int32_t kernel, double* ms, int64_t* launches) {
  if (kernel < 0 || kernel > 2) return fail(LDPC_FD_E_INVALID, "unknown kernel id");
  double total = 0.0;
  int64_t n = 0;
  for (auto& pr : t_prof.ev[kernel]) {
    HIP_TRY(hipEventSynchronize(pr.second));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
    total += t;
    ++n;
    t_prof.pool.push_back(pr.first);
    t_prof.pool.push_back(pr.second);
  }
  t_prof.ev[kernel].clear();
  if (ms) *ms = total;
  if (launches) *launches = n;
  return LDPC_FD_OK;
}

}  // extern "C"

#include "pool.inc"
#include "posterior.inc"

// ===========================================================================
// Decode with the argument struct and flags, several rounds from an imported
// state, and a pool sized from an HBM budget.
extern "C" {

int32_t ldpc_fd_decode_ex(ldpc_fd_code c, const ldpc_fd_decode_args* a, void* stream) {
  if (!c || !a) return fail(LDPC_FD_E_INVALID, "NULL code or arguments");
  const uint32_t known = LDPC_FD_FLAG_NO_EARLY_STOP | LDPC_FD_FLAG_VALIDATION | LDPC_FD_FLAG_ASYNC;
  if (a->flags & ~known) return fail(LDPC_FD_E_INVALID, "unknown flag bits");
  if (a->frames > 0 && !a->llr) return fail(LDPC_FD_E_INVALID, "NULL buffer");
  const bool val = (a->flags & LDPC_FD_FLAG_VALIDATION) != 0;
  if (val && a->mode != LDPC_FD_MODE_FUSED)
    return fail(LDPC_FD_E_UNSUPPORTED, "validation posteriors follow a FUSED decode");
  if (val && a->frames > 0 && !a->posterior) return fail(LDPC_FD_E_INVALID, "VALIDATION needs a posterior buffer");
  int32_t rc = decode_impl(c, a->frames, a->llr, nullptr, a->max_iter, a->prec, a->mode, a->hard, a->synd, a->iters,
                           a->status, a->workspace, a->workspace_bytes, stream, a->flags);
  if (rc || !val || a->frames == 0) return rc;
  return ldpc_fd_decode_posterior(c, a->frames, a->llr, a->prec, a->iters, a->workspace, a->workspace_bytes,
                                  a->posterior, stream);
}

int32_t ldpc_fd_run_rounds(ldpc_fd_code c, int32_t F, const float* llr, int32_t rounds, int32_t from_channel,
                           float* c2v_inout, uint8_t* hard, uint8_t* fsynd, uint8_t* synd, int32_t mode, int32_t prec,
                           void* stream) {
  if (!c) return fail(LDPC_FD_E_INVALID, "code is NULL");
  if (rounds < 1 || rounds > 100000) return fail(LDPC_FD_E_INVALID, "rounds outside 1..100000");
  if (!c2v_inout && F > 0) return fail(LDPC_FD_E_INVALID, "NULL c2v_inout");
  const bool decides = !from_channel || rounds > 1;
  int32_t rc = round_check(c, F, llr, decides ? c2v_inout : nullptr, mode == LDPC_FD_MODE_FUSED ? nullptr : c2v_inout,
                           c2v_inout, hard, fsynd, synd, mode, prec);
  if (rc || F == 0) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t msg = align256((size_t)F * c->E * c->q * 4);
  const size_t tmp_bytes = round_layout(c, F, prec, nullptr, nullptr);
  char* mem = nullptr;
  HIP_TRY(hipMalloc((void**)&mem, 2 * msg + tmp_bytes));
  float* other = (float*)mem;                 // the state of the alternate rounds
  float* v2c = (float*)(mem + msg);           // variable-to-check messages (PLAIN, LOGSP, FSP)
  char* tmp = mem + 2 * msg;
  float* cur = c2v_inout;
  float* nxt = other;
  for (int r = 0; r < rounds && rc == LDPC_FD_OK; ++r) {
    const float* in = (r == 0 && from_channel) ? nullptr : cur;
    rc = round_impl(c, F, llr, in, mode == LDPC_FD_MODE_FUSED ? nullptr : v2c, nxt, hard, fsynd, synd, mode, prec, s,
                    tmp);
    std::swap(cur, nxt);
  }
  // the last round's output is in `cur`
  if (rc == LDPC_FD_OK && cur != c2v_inout)
    rc = hipMemcpyAsync(c2v_inout, cur, (size_t)F * c->E * c->q * 4, hipMemcpyDeviceToDevice, s) == hipSuccess
             ? LDPC_FD_OK
             : fail(LDPC_FD_E_HIP, "hipMemcpyAsync");
  hipError_t e1 = hipStreamSynchronize(s);
  hipError_t e2 = hipFree(mem);
  if (rc) return rc;
  if (e1 != hipSuccess) return fail(LDPC_FD_E_HIP, std::string("run_rounds: ") + hipGetErrorString(e1));
  if (e2 != hipSuccess) return fail(LDPC_FD_E_HIP, std::string("hipFree: ") + hipGetErrorString(e2));
  return LDPC_FD_OK;
}

int32_t ldpc_fd_pool_budget_slots(const ldpc_fd_code* codes, int32_t ncodes, int64_t hbm_budget, int32_t prec,
                                  int32_t* slots) {
  if (!codes || ncodes < 1 || ncodes > 16) return fail(LDPC_FD_E_INVALID, "1..16 codes required");
  if (!slots) return fail(LDPC_FD_E_INVALID, "slots is NULL");
  if (prec < 0 || prec > 2) return fail(LDPC_FD_E_INVALID, "unknown precision");
  if (hbm_budget < 1) return fail(LDPC_FD_E_INVALID, "budget must be positive");
  const int64_t share = hbm_budget / ncodes;
  for (int k = 0; k < ncodes; ++k) {
    if (!codes[k]) return fail(LDPC_FD_E_INVALID, "NULL code");
    const int64_t per = (int64_t)pool_slot_bytes(codes[k], prec);
    const int64_t n = share / per;
    if (n < 1)
      return fail(LDPC_FD_E_NOMEM, "the budget's share of code " + std::to_string(k) + " holds no frame slot (" +
                                       std::to_string(per) + " bytes each)");
    slots[k] = (int32_t)std::min<int64_t>(n, 1 << 22);
  }
  return LDPC_FD_OK;
}

int32_t ldpc_fd_pool_create_budget(const ldpc_fd_code* codes, int32_t ncodes, int64_t hbm_budget, int32_t prec,
                                   void* stream, ldpc_fd_pool* out) {
  if (!out) return fail(LDPC_FD_E_INVALID, "out is NULL");
  *out = nullptr;
  std::vector<int32_t> slots(std::max(ncodes, 1));
  const int32_t rc = ldpc_fd_pool_budget_slots(codes, ncodes, hbm_budget, prec, slots.data());
  if (rc) return rc;
  return ldpc_fd_pool_create(codes, ncodes, slots.data(), prec, stream, out);
}

}  // extern "C"
