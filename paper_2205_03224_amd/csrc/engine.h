// Host-side engine interface of libgemslr (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "gs_internal.h"

namespace gs {

void hipcheck(hipError_t e, const char* what);
double now_s();

// Device allocations owned by one object, released together.
struct DevMem {
  std::vector<void*> ptrs;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem();
  void* raw(size_t bytes);
  template <class U> U* alloc(size_t n) { return (U*)raw(n * sizeof(U)); }
};

// Level-scheduled stage layout of one triangle of one level (host copy).
template <class T>
struct TriHost {
  std::vector<int32_t> blk_stage{0}, stage_row{0}, stage_ent{0};
  std::vector<uint32_t> rowinfo;
  std::vector<T> dinv, val;
  std::vector<uint16_t> col;
  int maxslot = 0, depth = 0;
  int maxwidth = 0;  // most rows in one wavefront level (stage) of one block
  // streamed layout only: per row slot, how many of its stored entries (the
  // last ones) refer to rows of the stage just before
  std::vector<uint8_t> nnear;
};
template <class T>
TriHost<T> build_tri(const CSR<T>& M, const std::vector<int64_t>& blocks, bool upper);
template <class T>
TriHost<T> build_tri_sched(const CSR<T>& M, const std::vector<int64_t>& blocks, bool upper,
                           int width, int near_cap);

// The preconditioner on the device in one storage precision.  Vectors at
// this interface hold float64 (real) or complex128 values.
struct Engine {
  virtual ~Engine() = default;
  // y = M^{-1} x; permuted: x, y already in the reordered numbering
  virtual void apply(const void* x, void* y, bool permuted) = 0;
  // out = Ĝ_l v (s_l entries each)
  virtual void ghat(int l, const void* v, void* out) = 0;
  // the same for m vectors of s_l entries stored one after another, every
  // launch of a level covering all m (columns equal those of ghat)
  virtual void ghat_batch(int l, int m, const void* v, void* out) = 0;
  // y = M^{-1} x for m vectors of n entries stored one after another
  // (original ordering), every launch of a level covering all m (columns
  // equal those of apply)
  virtual void apply_batch(int m, const void* x, void* y) = 0;
  // install W_l (s_l x k) and H_l (k x k), host arrays of the value type
  virtual void set_lowrank(int l, int k, const void* W, const void* H) = 0;
  // the same with W_l in device memory (value type, s_l x k column-major,
  // read before the call returns): 1 when the engine now holds W_l exactly,
  // 0 when it holds it rounded to its storage type
  virtual int set_lowrank_device(int l, int k, const void* W, const void* H) = 0;
  // copy the installed W_l to host memory (value type); false when the
  // engine stores it in another precision
  virtual bool get_lowrank_w(int l, void* W) = 0;
  virtual void stats(gs_info* info, int vb_vec) = 0;
  virtual double bytes_per_apply() const = 0;
  // One apply per rep with HIP events around every launch; returns the number
  // of launches and, per launch, mean ms, compulsory bytes and a label.
  virtual int profile(const void* x, void* y, int reps, std::vector<double>& ms,
                      std::vector<double>& bytes, std::vector<std::string>& labels) = 0;
  // Bracket every later launch of kernel class `kind` with HIP events (up to
  // max_launches); probe_read synchronises and returns count, ms and bytes.
  virtual void probe_enable(int kind, int max_launches) = 0;
  virtual void probe_read(int64_t* launches, double* ms, double* bytes) = 0;
  // m > 0: m inner GMRES steps on S_hat_0 at the root level of every apply
  // (float64 / complex128 forms only); 0 switches them off
  virtual void set_inner(int m) = 0;
  // Device scratch one apply needs (working vector, partial sums and the
  // staging vectors of the levels that use them) when every buffer is cut
  // from one region at 256-byte offsets; 0 when the apply cannot run that
  // way (inner GMRES steps keep their own work space).
  virtual size_t scratch_bytes() const = 0;
  // apply(x, y, false) with every scratch buffer cut from `base`
  // (scratch_bytes() bytes, device memory, 256-byte aligned): no allocation.
  virtual void apply_in(const void* x, void* y, void* base) = 0;
};

// kernel classes for the measurement probe
enum { KIND_TRI0 = 0, KIND_TRI = 1, KIND_INTERFACE = 2, KIND_LOWRANK = 3, KIND_PERM = 4 };

std::unique_ptr<Engine> make_engine(const HostSetup<double>& S, int precision, hipStream_t st);
std::unique_ptr<Engine> make_engine(const HostSetup<cplx>& S, int precision, hipStream_t st);

}  // namespace gs
