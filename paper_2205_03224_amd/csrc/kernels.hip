// HIP kernels of libgemslr for gfx950 (CDNA4, 64-wide wavefronts).
//
// The preconditioner apply (Alg. 2) is a chain of bandwidth-bound sparse
// steps; every kernel below streams its operands once, with the 64 lanes of
// a wavefront reading consecutive addresses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cstdlib>

#include "device.h"

namespace gs {

namespace {

constexpr int kWave = 64;

template <class T> __device__ inline T zero();
template <class T> __device__ inline T cvt_rc(float v);
template <> __device__ inline double cvt_rc<double>(float v) { return (double)v; }
template <> __device__ inline dcplx cvt_rc<dcplx>(float v) { return mk((double)v, 0.0); }
template <> __device__ inline double zero<double>() { return 0.0; }
template <> __device__ inline float zero<float>() { return 0.0f; }
template <> __device__ inline dcplx zero<dcplx>() { return mk(0.0, 0.0); }

// c ? a : b, component-wise for complex values (a select of the struct as
// a whole is lowered through scratch memory)
__device__ inline double sel(bool c, double a, double b) { return c ? a : b; }
__device__ inline float sel(bool c, float a, float b) { return c ? a : b; }
__device__ inline dcplx sel(bool c, dcplx a, dcplx b) { return mk(c ? a.x : b.x, c ? a.y : b.y); }

// Fixed-order sums over the 256 threads of a workgroup through LDS (two
// read rounds; a shuffle chain costs one LDS round trip per step).
// block_sum8: thread c < 8 gets the sum of every thread's v[c]; red holds
// 9 x 256 values.  block_sum1: thread 0 gets the sum of v; red holds 288.
// Both end with a barrier, so red may be reused right after.
constexpr int kRedThreads = 256;
template <class T>
__device__ inline T block_sum8(const T (&v)[8], T* red, int tid) {
#pragma unroll
  for (int u = 0; u < 8; ++u) red[u * kRedThreads + tid] = v[u];
  __syncthreads();
  {
    const int u = tid / 32, g = tid % 32;
    T s = zero<T>();
#pragma unroll
    for (int i = 0; i < 8; ++i) s += red[u * kRedThreads + g * 8 + i];
    red[8 * kRedThreads + tid] = s;
  }
  __syncthreads();
  T r = zero<T>();
  if (tid < 8)
    for (int g = 0; g < 32; ++g) r += red[8 * kRedThreads + tid * 32 + g];
  __syncthreads();
  return r;
}
template <class T>
__device__ inline T block_sum1(T v, T* red, int tid) {
  red[tid] = v;
  __syncthreads();
  if (tid < 32) {
    T s = zero<T>();
#pragma unroll
    for (int i = 0; i < 8; ++i) s += red[tid * 8 + i];
    red[kRedThreads + tid] = s;
  }
  __syncthreads();
  T r = zero<T>();
  if (tid == 0)
    for (int g = 0; g < 32; ++g) r += red[kRedThreads + g];
  __syncthreads();
  return r;
}

// r[u] = sum_p val[p] * x[ci[p]] over the CSR rows row[u] (row < 0: none)
// of one thread, with every row's entries fetched together: row pointers,
// then up to B entries of every row (indices and values), then the gathers.
// A row of length n costs ceil(n / B) rounds, all rows at once.
// IDX: x is indexed by the entry itself (x[p], values already gathered in
// entry order), ci unused.
template <class C, class VT, class XT, int U, int B, bool IDX = false>
__device__ __forceinline__ void csr_rows(const int32_t* rp, const int32_t* ci, const VT* val,
                                         const XT* x, const int (&row)[U], C (&r)[U]) {
  int p0[U], p1[U];
  int mx = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    p0[u] = row[u] >= 0 ? rp[row[u]] : 0;
    p1[u] = row[u] >= 0 ? rp[row[u] + 1] : 0;
    r[u] = zero<C>();
  }
#pragma unroll
  for (int u = 0; u < U; ++u) mx = max(mx, p1[u] - p0[u]);
  for (int m = 0; m < mx; m += B) {  // mx > 0 implies at least one entry exists
    int cc[U][B];
    C fv[U][B];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < B; ++t) {
        const int q = p0[u] + m + t;
        const bool ok = q < p1[u];
        const int qq = ok ? q : 0;
        cc[u][t] = IDX ? qq : ci[qq];
        fv[u][t] = sel(ok, cvt<C>(val[qq]), zero<C>());
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < B; ++t) r[u] += fv[u][t] * cvt<C>(x[cc[u][t]]);
  }
}

}  // namespace

// ======================================================================
// Batched block triangular solve: one wavefront per diagonal block.
//
// For block b the wavefront loads its right-hand side into LDS, runs the
// forward sweep with L (unit diagonal) and the backward sweep with U over
// the level-scheduled stages, and writes the result.  Rows of one stage are
// independent, so each lane owns one row; stages follow each other in
// dependency order and only LDS carries values between them, in program
// order of the single wavefront (no barrier needed).  The factor entries of
// the next stage are fetched into registers while the current stage
// computes, so HBM latency overlaps the dependent LDS chain.
//
// MODE TRI_DOWN: rhs = t[rows], result stored to t[rows]           (z1)
// MODE TRI_UP:   rhs = F_l y2 (y2 = t[d ...]), t[rows] -= result   (y1)
// ======================================================================

template <class P, int MS>
struct StageRegs {
  typename P::C v[MS > 0 ? MS : 1];
  uint16_t c[MS > 0 ? MS : 1];
  uint32_t info;
  typename P::C dinv;
};

template <class P, int MS, bool ISU>
__device__ __forceinline__ void stage_load(const TriDev<P>& tri, int s, int lane,
                                           StageRegs<P, MS>& r) {
  using C = typename P::C;
  const int r0 = tri.stage_row[s];
  const int nrs = tri.stage_row[s + 1] - r0;
  int e = tri.stage_ent[s];
  const bool act = lane < nrs;
  r.info = act ? tri.rowinfo[r0 + lane] : 0u;
  const int nz = (int)(r.info >> 16);
  const int maxnz = __builtin_amdgcn_readfirstlane(nz);
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    if (j < maxnz) {
      const unsigned long long m = __ballot(nz > j);
      if (nz > j) {
        r.v[j] = cvt<C>(tri.val[e + lane]);
        r.c[j] = tri.col[e + lane];
      }
      e += __popcll(m);
    }
  }
  if (ISU) r.dinv = sel(act, cvt<C>(tri.dinv[r0 + lane]), zero<C>());
}

template <class P, int MS, bool ISU>
__device__ __forceinline__ void stage_compute(const StageRegs<P, MS>& r,
                                              typename P::C* x) {
  using C = typename P::C;
  const int nz = (int)(r.info >> 16);
  const int row = (int)(r.info & 0xffffu);
  const int maxnz = __builtin_amdgcn_readfirstlane(nz);
  // all gathers first (masked slots read x[row]), then the accumulation
  C xv[MS > 0 ? MS : 1];
#pragma unroll
  for (int j = 0; j < MS; ++j)
    if (j < maxnz) xv[j] = x[nz > j ? (int)r.c[j] : row];
  C acc = x[row];
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    if (j < maxnz) {
      const C t = r.v[j] * xv[j];
      acc = sel(nz > j, acc - t, acc);
    }
  }
  if (ISU) acc *= r.dinv;
  x[row] = acc;
}

// generic path for rows longer than the register budget: entries are read
// as they are used
template <class P, bool ISU>
__device__ void sweep_generic(const TriDev<P>& tri, int s0, int s1, int lane,
                              typename P::C* x, bool sync) {
  using C = typename P::C;
  for (int s = s0; s < s1; ++s) {
    const int r0 = tri.stage_row[s];
    const int nrs = tri.stage_row[s + 1] - r0;
    int e = tri.stage_ent[s];
    const bool act = lane < nrs;
    const uint32_t info = act ? tri.rowinfo[r0 + lane] : 0u;
    const int nz = (int)(info >> 16);
    const int maxnz = __builtin_amdgcn_readfirstlane(nz);
    C acc = sel(act, x[info & 0xffffu], zero<C>());
    for (int j = 0; j < maxnz; ++j) {
      const unsigned long long m = __ballot(nz > j);
      if (nz > j) acc -= cvt<C>(tri.val[e + lane]) * x[tri.col[e + lane]];
      e += __popcll(m);
    }
    if (act) {
      if (ISU) acc *= cvt<C>(tri.dinv[r0 + lane]);
      x[info & 0xffffu] = acc;
    }
    if (sync) __syncthreads();
  }
}

template <class P, int MS, bool ISU>
__device__ __forceinline__ void sweep(const TriDev<P>& tri, int s0, int s1, int lane,
                                      typename P::C* x, bool sync) {
  if (MS == 0) {
    sweep_generic<P, ISU>(tri, s0, s1, lane, x, sync);
    return;
  }
  if (s0 >= s1) return;
  StageRegs<P, MS> A, B;
  stage_load<P, MS, ISU>(tri, s0, lane, A);
  for (int s = s0; s < s1; s += 2) {
    if (s + 1 < s1) stage_load<P, MS, ISU>(tri, s + 1, lane, B);
    if (lane < tri.stage_row[s + 1] - tri.stage_row[s]) stage_compute<P, MS, ISU>(A, x);
    if (sync) __syncthreads();
    if (s + 1 >= s1) break;
    if (s + 2 < s1) stage_load<P, MS, ISU>(tri, s + 2, lane, A);
    if (lane < tri.stage_row[s + 2] - tri.stage_row[s + 1]) stage_compute<P, MS, ISU>(B, x);
    if (sync) __syncthreads();
  }
}

template <class P, int MS, bool XLDS, int MODE>
__global__ __launch_bounds__(64) void k_trisolve(TriArgs<P> a) {
  using C = typename P::C;
  using X = typename P::X;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int r0 = a.blk_row[b];
  const int nr = a.blk_row[b + 1] - r0;
  C* x = XLDS ? reinterpret_cast<C*>(smem_raw) : reinterpret_cast<C*>(a.xg) + r0;
  // right-hand side
  for (int i = lane; i < nr; i += kWave) {
    C r;
    if (MODE == TRI_DOWN) {
      r = cvt<C>(a.t[r0 + i]);
    } else {
      r = zero<C>();
      const int p0 = a.F.rp[r0 + i], p1 = a.F.rp[r0 + i + 1];
      for (int p = p0; p < p1; ++p) r += cvt<C>(a.F.v[p]) * cvt<C>(a.t[a.d + a.F.ci[p]]);
    }
    x[i] = r;
  }
  if (!XLDS) __syncthreads();
  sweep<P, MS, false>(a.lo, a.lo.blk_stage[b], a.lo.blk_stage[b + 1], lane, x, !XLDS);
  sweep<P, MS, true>(a.up, a.up.blk_stage[b], a.up.blk_stage[b + 1], lane, x, !XLDS);
  for (int i = lane; i < nr; i += kWave) {
    if (MODE == TRI_DOWN) a.t[r0 + i] = cvt<X>(x[i]);
    else a.t[r0 + i] = cvt<X>(cvt<C>(a.t[r0 + i]) - x[i]);
  }
}

template <class P, int MS, int MODE>
static void launch_tri_ms(const TriArgs<P>& a, int max_block_rows, hipStream_t st) {
  using C = typename P::C;
  const size_t lds = (size_t)max_block_rows * sizeof(C);
  if (lds <= 65536) {
    hipLaunchKernelGGL((k_trisolve<P, MS, true, MODE>), dim3(a.nb), dim3(kWave), lds, st, a);
  } else {
    hipLaunchKernelGGL((k_trisolve<P, MS, false, MODE>), dim3(a.nb), dim3(kWave), 0, st, a);
  }
}

template <class P, int MODE>
static void launch_tri_mode(const TriArgs<P>& a, int maxslot, int mbr, hipStream_t st) {
  if (maxslot <= 4) launch_tri_ms<P, 4, MODE>(a, mbr, st);
  else if (maxslot <= 8) launch_tri_ms<P, 8, MODE>(a, mbr, st);
  else if (maxslot <= 12) launch_tri_ms<P, 12, MODE>(a, mbr, st);
  else if (maxslot <= 16) launch_tri_ms<P, 16, MODE>(a, mbr, st);
  else launch_tri_ms<P, 0, MODE>(a, mbr, st);
}

template <class P>
void launch_trisolve(const TriArgs<P>& a0, int mode, int maxslot, int max_block_rows,
                     hipStream_t st) {
  if (a0.nb <= 0) return;
  // several vectors: one launch each (they share the global block-vector
  // staging, in stream order)
  for (int j = 0; j < a0.nvec; ++j) {
    TriArgs<P> a = a0;
    a.t += (int64_t)j * a0.ldt;
    a.fy += (int64_t)j * a0.ldfy;
    a.nvec = 1;
    if (mode == TRI_DOWN) launch_tri_mode<P, TRI_DOWN>(a, maxslot, max_block_rows, st);
    else launch_tri_mode<P, TRI_UP>(a, maxslot, max_block_rows, st);
  }
}

// ======================================================================
// Streamed batched block triangular solve: two wavefronts per diagonal
// block.  Wave 1 (producer) copies the block's chunks -- whole stages of
// factor entries, row info and inverse diagonals, packed contiguously --
// from HBM into one of two LDS buffers with 16-byte coalesced loads, while
// wave 0 (consumer) runs the dependent sweep over the other buffer out of
// LDS only.  One workgroup barrier per chunk hands the buffers over.  HBM
// latency is paid once per chunk instead of once per wavefront level.
// ======================================================================

// n16 > 0 units of 16 bytes from src to LDS dst by one wave, as described
// below for copy_chunk
__device__ __forceinline__ void copy_to_lds(const uint4* src, int n16, uint8_t* dst, int lane,
                                            int iters) {
  const int last = n16 - 1;
  for (int i = 0; i < iters; ++i)
    __builtin_amdgcn_global_load_lds(src + min(lane + kWave * i, last),
                                     (__attribute__((address_space(3))) void*)(dst + 1024 * i),
                                     16, 0, 0);
}
template <class P>
__device__ __forceinline__ void copy_chunk(const TriArgs<P>& a, const ChunkDesc& cd, uint8_t* dst,
                                           int lane, int iters) {
  // Direct HBM -> LDS copies (global_load_lds, 16 bytes per lane): iteration
  // i fills dst[1 KiB i, 1 KiB (i+1)), lane l its 16 bytes at 16 l.  The
  // loads carry no register data and no wait, so the whole chunk is in flight
  // at once.  Lanes past the end re-read the last 16 bytes and land behind
  // the chunk, inside the buffer (iters * 1 KiB <= chunk_cap, a multiple of
  // 1 KiB); a caller may ask for more iterations than the chunk needs.
  copy_to_lds(reinterpret_cast<const uint4*>(a.blob + cd.off), (int)cd.n16, dst, lane, iters);
}

// s_waitcnt immediates (vmcnt n; expcnt and lgkmcnt at their maxima)
#define GS_VMCNT_IMM(n) (((n) & 15) | (((n) >> 4) << 14) | 0x0F70)

// Chunk descriptors of a block held in registers, lane j holding chunk
// base + j: reading one is a lane read, not a memory load.  (A per-chunk
// global load would put its latency on the consumer's path, and on the
// producer's it would wait behind the copies in flight, since vector-memory
// loads complete in order.)  Refilled once per 64 chunks.
struct DescCache {
  uint32_t w[4];
  int base;
};
template <class P>
__device__ __forceinline__ void desc_fill(const TriArgs<P>& a, int first, int c1, int lane,
                                          DescCache& d) {
  const uint4 v = reinterpret_cast<const uint4*>(a.chunk)[min(first + lane, c1 - 1)];
  // wait here, inside the refill, so that no wait is left pending on the
  // common path (vector-memory loads complete in order: a wait outside
  // would also wait for the copies in flight)
  __builtin_amdgcn_s_waitcnt(GS_VMCNT_IMM(0));
  d.w[0] = v.x;
  d.w[1] = v.y;
  d.w[2] = v.z;
  d.w[3] = v.w;
  d.base = __builtin_amdgcn_readfirstlane(first);
}
template <class P>
__device__ __forceinline__ ChunkDesc desc_get(const TriArgs<P>& a, int c, int c1, int lane,
                                              DescCache& d) {
  static_assert(sizeof(ChunkDesc) == 16, "ChunkDesc is four words");
  if (c - d.base >= kWave) desc_fill<P>(a, c, c1, lane, d);
  const int j = c - d.base;
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) w[q] = (uint32_t)__builtin_amdgcn_readlane((int)d.w[q], j);
  ChunkDesc cd;
  __builtin_memcpy(&cd, w, sizeof(cd));
  return cd;
}

// lgkmcnt(0) alone (vmcnt and expcnt at their maxima)
#define GS_LGKM0_IMM 0xC07F

// the partner lane's (lane +- 32) value of x
__device__ __forceinline__ double swap32(double x, bool low) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)(low ? b[1] : b[0]), (int)(low ? a[1] : a[0]));
}
__device__ __forceinline__ float swap32(float x, bool low) {
  const unsigned u = __float_as_uint(x);
  const auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return __uint_as_float(low ? a[1] : a[0]);
}
__device__ __forceinline__ dcplx swap32(dcplx x, bool low) {
  return mk(swap32(x.x, low), swap32(x.y, low));
}

// Lanes 0..31 receive the value of x in lane + 32 (returned in `hi`) while
// keeping their own (returned in `lo`); `dead` is a value the caller no
// longer needs (the swap overwrites its register), so no copies are made.
// Lanes 32..63 get unspecified values.
__device__ __forceinline__ void from_high(double x, double dead, double& lo, double& hi) {
  const auto a = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x),
                                                  (unsigned)__double2loint(dead), false, false);
  const auto b = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x),
                                                  (unsigned)__double2hiint(dead), false, false);
  lo = __hiloint2double((int)b[0], (int)a[0]);
  hi = __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ void from_high(float x, float dead, float& lo, float& hi) {
  const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(dead), false,
                                                  false);
  lo = __uint_as_float(a[0]);
  hi = __uint_as_float(a[1]);
}
__device__ __forceinline__ void from_high(dcplx x, dcplx dead, dcplx& lo, dcplx& hi) {
  from_high(x.x, dead.x, lo.x, hi.x);
  from_high(x.y, dead.y, lo.y, hi.y);
}

// Pipeline over the stages of one chunk (full rows, or half rows: lanes l
// and l + 32 share row l).  A lane's SL slots split into NF far slots, whose
// columns were computed two or more stages back, and the NN near slots after
// them, which may refer to the stage just before (near_slots; the layout
// guarantees the split).  Per stage s:
//   1. gather the near slots of s -- LDS executes one wavefront's accesses
//      in order, so these see the store of s - 1 that precedes them;
//   2. form the gather addresses of s + 1 and gather its far slots and the
//      current value of its rows (nothing of stage s is involved);
//   3. issue the loads of s + 2 (entries, columns, 1/u_ii, the row info of
//      s + 3), ahead of the near wait when the LDS counter can still tell the
//      near gathers apart (at most 15 operations younger), else after it;
//   4. add the far products of s (gathered during stage s - 1);
//   5. add the near products, finish and store the result of s.
// So the critical path of a stage is the store -> near-gather round trip plus
// NN products and the finish, and the far gathers and loads travel while the
// previous stage completes.  Scheduling barriers keep the order; the compiler
// places the waits at the first use of each gathered value.
template <class P, int MS, bool HALF>
struct PipeRegs {
  using C = typename P::C;
  static constexpr int SL = HALF ? MS / 2 : MS;  // slots per lane
  static constexpr int NN = near_slots(MS, HALF);
  static constexpr int NF = SL - NN;
  static constexpr int NW = (SL + 1) / 2;        // 32-bit words of packed columns
  C v[SL];
  uint32_t cw[NW];
  uint32_t ad[SL];  // gather byte offsets into the block vector
  C dv;
  uint32_t row;  // LDS byte offset of the lane's row in the block vector, or
                 // of the dummy slot (idle lanes; in half rows the high lane)
  int nr;   // rows of the stage (uniform; 0 past the chunk's last stage)
  C xv[SL];  // gathered block-vector values
  C b;       // current value of the row (right-hand side)
};

// load of a value at LDS byte address a
template <class C>
__device__ __forceinline__ C lds_ld(uint32_t a) {
  typedef __attribute__((address_space(3))) const C T;
  return *(T*)(size_t)a;
}
template <>
__device__ __forceinline__ dcplx lds_ld<dcplx>(uint32_t a) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(3))) const d2 T;
  const d2 v = *(T*)(size_t)a;
  return mk(v.x, v.y);
}

template <>
__device__ __forceinline__ bf16 lds_ld<bf16>(uint32_t a) {
  typedef __attribute__((address_space(3))) const uint16_t T;
  return bf16{*(T*)(size_t)a};
}

// store of a value at LDS byte address a
template <class C>
__device__ __forceinline__ void lds_st(uint32_t a, C v) {
  typedef __attribute__((address_space(3))) C T;
  *(T*)(size_t)a = v;
}
template <>
__device__ __forceinline__ void lds_st<dcplx>(uint32_t a, dcplx v) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(3))) d2 T;
  d2 w;
  w.x = v.x;
  w.y = v.y;
  *(T*)(size_t)a = w;
}

// LDS byte address of a block-vector element (x0: LDS address of x[0])
template <class P, int MS, bool HALF>
__device__ __forceinline__ void st_addr(PipeRegs<P, MS, HALF>& R, uint32_t x0) {
  using C = typename P::C;
  constexpr int kMul = (int)sizeof(C) / ColScale<C>::value;
#pragma unroll
  for (int j = 0; j < PipeRegs<P, MS, HALF>::SL; ++j) {
    R.ad[j] = x0 + (j % 2 ? R.cw[j / 2] >> 16 : R.cw[j / 2] & 0xffffu) * kMul;
    asm volatile("" : "+v"(R.ad[j]));  // formed here, not again before the gathers
  }
}

// loads of one stage whose row info is `info` and first chunk row r0; the
// chunk's sections are given by LDS byte addresses (32-bit arithmetic)
template <class P, int MS, bool HALF, bool ISU>
__device__ __forceinline__ void st_load(uint32_t vbase, uint32_t dbase, uint32_t cbase,
                                        uint32_t info, int r0, int ql, int half, int dummy,
                                        PipeRegs<P, MS, HALF>& R) {
  using C = typename P::C;
  using V = typename P::V;
  using D = typename P::D;
  using RG = PipeRegs<P, MS, HALF>;
  constexpr int VS = stream_vstride(MS), CS = stream_cstride(MS);
  constexpr int CO = HALF ? stream_half_coff(MS) : 0;
  static_assert(CO + RG::SL <= CS, "column row holds both halves");
  R.nr = (int)__builtin_amdgcn_readfirstlane(info >> 24);
  const bool act = ql < R.nr;
  R.row = (act && (!HALF || half == 0)) ? (info & 0xffffffu) : (uint32_t)dummy;
  const uint32_t q = (uint32_t)(act ? r0 + ql : r0);
  const uint32_t va = vbase + __umul24(q, (uint32_t)(VS * sizeof(V))) +
                      (HALF ? (uint32_t)(half * RG::SL * sizeof(V)) : 0u);
  const uint32_t ca = cbase + __umul24(q, (uint32_t)(CS * 2)) + (HALF ? (uint32_t)(half * CO * 2) : 0u);
#pragma unroll
  for (int j = 0; j < RG::SL; ++j) R.v[j] = cvt<C>(lds_ld<V>(va + j * (uint32_t)sizeof(V)));
#pragma unroll
  for (int j = 0; j < RG::NW; ++j) R.cw[j] = lds_ld<uint32_t>(ca + 4u * j);
  if (ISU) R.dv = cvt<C>(lds_ld<D>(dbase + q * (uint32_t)sizeof(D)));
}

// gathers of slots J0 .. J1 - 1
template <int J0, int J1, class P, int MS, bool HALF>
__device__ __forceinline__ void st_gather(PipeRegs<P, MS, HALF>& R) {
  using C = typename P::C;
#pragma unroll
  for (int j = J0; j < J1; ++j) R.xv[j] = lds_ld<C>(R.ad[j]);
}
// current value of the lane's row
template <class P, int MS, bool HALF>
__device__ __forceinline__ void st_gather_b(PipeRegs<P, MS, HALF>& R, uint32_t x0) {
  using C = typename P::C;
  R.b = lds_ld<C>(x0 + R.row);
}

// the two partial sums (even and odd slots; padded entries are zero)
template <class C>
struct PipeAcc {
  C s0, s1;
};
template <int J0, int J1, class P, int MS, bool HALF>
__device__ __forceinline__ void st_sum(const PipeRegs<P, MS, HALF>& R, PipeAcc<typename P::C>& a) {
#pragma unroll
  for (int j = J0; j < J1; ++j) {
    if (j % 2 == 0) a.s0 += R.v[j] * R.xv[j];
    else a.s1 += R.v[j] * R.xv[j];
  }
}

// x[row] = (b - sum_j v_j x[c_j]) (* 1/u_ii); half rows: the low lane adds
// its half sum and the high lane's, in that order (the high lane stores to
// the dummy slot)
template <class P, int MS, bool HALF, bool ISU>
__device__ __forceinline__ void st_finish(const PipeRegs<P, MS, HALF>& R,
                                          const PipeAcc<typename P::C>& a, uint32_t x0) {
  using C = typename P::C;
  C acc;
  if (HALF) {
    C p, o;
    from_high(a.s0 + a.s1, a.s1, p, o);
    acc = R.b - (p + o);
  } else {
    acc = R.b - (a.s0 + a.s1);
  }
  if (ISU) acc *= R.dv;
  lds_st<C>(x0 + R.row, acc);
}

template <class P, int MS, bool HALF, bool ISU>
__device__ __forceinline__ void chunk_sweep(const uint8_t* cb, const ChunkDesc& cd, int lane,
                                            typename P::C* x, int dummy) {
  using C = typename P::C;
  using V = typename P::V;
  using RG = PipeRegs<P, MS, HALF>;
  constexpr int SL = RG::SL, NF = RG::NF, NW = RG::NW;
  // LDS operations of one stage's loads (paired where adjacent) and of the
  // far gathers; the loads go ahead of the near wait when the near gathers
  // stay within the 15 operations the counter tells apart
  constexpr int kLoadOps = (SL * (int)sizeof(V) + 15) / 16 + (NW + 1) / 2 + (ISU ? 2 : 1);
  constexpr bool kEarly = NF + 1 + kLoadOps <= 15;
  typedef __attribute__((address_space(3))) const uint8_t lds_u8;
  const uint32_t vbase = (uint32_t)(size_t)(lds_u8*)cb;
  const uint32_t dbase = vbase + 16u * cd.dinv16;
  const uint32_t ibase = vbase + 16u * cd.info16;
  const uint32_t cbase = vbase + 16u * cd.col16;
  const auto rinfo = [&](int i) { return lds_ld<uint32_t>(ibase + 4u * (uint32_t)i); };
  const int nst = cd.nst & 0x7fff;
  if (nst == 0) return;
  const int nrows = (int)cd.nrows;
  const int ql = HALF ? (lane & 31) : lane, half = HALF ? lane >> 5 : 0;
  typedef __attribute__((address_space(3))) C lds_c;
  const uint32_t x0 = (uint32_t)(size_t)(lds_c*)x;
  RG A, B, Cr;
  // prologue: stages 0 and 1 loaded, the row info of stage 2 read, the far
  // slots of stage 0 gathered (everything before the chunk is complete).
  // Row info read past the chunk's last stage is the closing zero word: a
  // stage of no rows.
  st_load<P, MS, HALF, ISU>(vbase, dbase, cbase, rinfo(ql), 0, ql, half, dummy, A);
  int r = A.nr;
  uint32_t info = rinfo(min(r + ql, nrows));
  st_load<P, MS, HALF, ISU>(vbase, dbase, cbase, info, r, ql, half, dummy, B);
  r += B.nr;
  info = rinfo(min(r + ql, nrows));
  st_addr<P, MS, HALF>(A, x0);
  st_gather<0, NF>(A);
  st_gather_b(A, x0);
  // one stage: cur = s, nxt = s+1, far receives s+2
  const auto step = [&](RG& cur, RG& nxt, RG& far, int s) {
    st_gather<NF, SL>(cur);
    __builtin_amdgcn_sched_barrier(0);
    st_addr<P, MS, HALF>(nxt, x0);
    st_gather<0, NF>(nxt);
    st_gather_b(nxt, x0);
    __builtin_amdgcn_sched_barrier(0);
    const auto loads = [&] {
      st_load<P, MS, HALF, ISU>(vbase, dbase, cbase, info, r, ql, half, dummy, far);
      r += far.nr;
      info = rinfo(min(r + ql, nrows));
    };
    if (kEarly) loads();
    __builtin_amdgcn_sched_barrier(0);
    PipeAcc<C> acc{zero<C>(), zero<C>()};
    st_sum<0, NF>(cur, acc);
    __builtin_amdgcn_sched_barrier(0);
    if (!kEarly) {
      st_sum<NF, SL>(cur, acc);
      __builtin_amdgcn_sched_barrier(0);
      loads();
      __builtin_amdgcn_sched_barrier(0);
    } else {
      st_sum<NF, SL>(cur, acc);
    }
    st_finish<P, MS, HALF, ISU>(cur, acc, x0);
    __builtin_amdgcn_sched_barrier(0);
  };
  for (int s = 0;; s += 3) {
    step(A, B, Cr, s);
    if (s + 1 >= nst) break;
    step(B, Cr, A, s + 1);
    if (s + 2 >= nst) break;
    step(Cr, A, B, s + 2);
    if (s + 3 >= nst) break;
  }
}

// Vector c and row i of flat index e = c * nr + i, nv vectors (inv = 1 / nr
// in float: the quotient is off by at most one for e < 2^22 nr, fixed by one
// step)
__device__ __forceinline__ void split_flat(int e, int nr, int nv, float inv, int& c, int& i) {
  if (nv == 1) {
    c = 0;
    i = e;
    return;
  }
  c = (int)((float)e * inv);
  i = e - c * nr;
  if (i < 0) {
    --c;
    i += nr;
  } else if (i >= nr) {
    ++c;
    i -= nr;
  }
}

// Right-hand sides of a block into LDS, vector c of the workgroup at
// x + c * xs: DOWN reads b1, UP reads F_l y2.  The nv * nr entries form one
// flat range with U loads per thread in flight at once (U = 32 float64
// values: a whole 4096-row block in one round trip with 128 threads).
template <class P, int MODE, int U>
__device__ __forceinline__ void load_rhs(const TriArgs<P>& a, int r0, int nr, int nv, int tid,
                                         int nt, typename P::C* x, int xs) {
  using C = typename P::C;
  const int tot = nv * nr;
  const float inv = 1.0f / (float)max(nr, 1);
  for (int e0 = tid; e0 < tot; e0 += nt * U) {
    C r[U];
    int dst[U];
    if (MODE == TRI_DOWN && a.xin) {
      // one vector (the caller's), read through the permutation: all
      // permutation loads first, then all vector loads (two round trips)
      int src[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        dst[u] = min(e0 + u * nt, tot - 1);
        src[u] = r0 + dst[u];
      }
      if (a.perm) {
#pragma unroll
        for (int u = 0; u < U; ++u) src[u] = a.perm[src[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = cvt<C>(a.xin[src[u]]);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int c, i;
        split_flat(min(e0 + u * nt, tot - 1), nr, nv, inv, c, i);
        dst[u] = c * xs + i;
        if (MODE == TRI_DOWN) r[u] = cvt<C>(a.t[(int64_t)c * a.ldt + r0 + i]);
        else r[u] = a.fy[(int64_t)c * a.ldfy + r0 + i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * nt < tot) x[dst[u]] = r[u];
  }
}

// Right-hand sides of the up sweep, F_l y2, from the unit's F records (rows
// without entries are zero): every row's entries are added from zero in
// stored order, the operations of k_fy, so the sums are the same.  The
// (vector, record) pairs form one flat range; U pairs per thread and four
// entries of each are in flight at once.  The zero fill is ordered before
// the records' stores by a bare barrier, so the producer's first chunk copy
// stays in flight.
template <class P, int U>
__device__ __forceinline__ void rhs_from_f(const TriArgs<P>& a, int b, int nv, int tid, int nt,
                                           typename P::C* x, int xs) {
  using C = typename P::C;
  using X = typename P::X;
  for (int e = tid; e < nv * xs; e += nt) x[e] = zero<C>();
  __builtin_amdgcn_s_waitcnt(GS_LGKM0_IMM);
  __builtin_amdgcn_s_barrier();
  const X* y2 = a.t + a.d;
  const int q0 = a.funit[b], q1 = a.funit[b + 1];
  const int nq = q1 - q0, tot = nv * nq;
  const float inv = 1.0f / (float)max(nq, 1);
  constexpr int J = 4;
  for (int eb = tid; eb < tot; eb += nt * U) {
    int q[U], dst[U];
    const X* yv[U];
    C r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int c, i;
      split_flat(min(eb + u * nt, tot - 1), nq, nv, inv, c, i);
      q[u] = q0 + i;
      dst[u] = c * xs + a.frow[q[u]];
      yv[u] = y2 + (int64_t)c * a.ldt;
      r[u] = zero<C>();
    }
    for (int j0 = 0; j0 < a.fw; j0 += J) {
      int cc[U][J];
      C fv[U][J];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int jj = 0; jj < J; ++jj) {
          const int j = min(j0 + jj, a.fw - 1);
          const int64_t e = (int64_t)j * a.nrec + q[u];
          cc[u][jj] = a.fcol[e];
          fv[u][jj] = sel(j0 + jj < a.fw, cvt<C>(a.fval[e]), zero<C>());
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int jj = 0; jj < J; ++jj) r[u] += fv[u][jj] * cvt<C>(yv[u][cc[u][jj]]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (eb + u * nt < tot) x[dst[u]] = r[u];
  }
}

// store that does not keep the line in L2: the sweep's results are read
// next by other kernels, mostly on other XCDs (measured: 1.3 us less per
// apply at 128^3 than plain stores)
template <class T>
__device__ __forceinline__ void st_out(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}
template <>
__device__ __forceinline__ void st_out<dcplx>(dcplx* p, dcplx v) {
  st_out(&p->x, v.x);
  st_out(&p->y, v.y);
}

// Results of a block from LDS: DOWN stores z1, UP stores z1 - (LU)^{-1} F y2.
template <class P, int MODE>
__device__ __forceinline__ void store_result(const TriArgs<P>& a, int r0, int nr, int nv, int tid,
                                             int nt, const typename P::C* x, int xs) {
  using C = typename P::C;
  using X = typename P::X;
  constexpr int U = 8;
  const int tot = nv * nr;
  const float inv = 1.0f / (float)max(nr, 1);
  for (int e0 = tid; e0 < tot; e0 += nt * U) {
    if (MODE == TRI_DOWN) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int c, i;
        split_flat(min(e0 + u * nt, tot - 1), nr, nv, inv, c, i);
        if (e0 + u * nt < tot) st_out(&a.t[(int64_t)c * a.ldt + r0 + i], cvt<X>(x[c * xs + i]));
      }
    } else if (a.yout) {
      // one vector: y1 = z1 - x straight to the caller's vector
      C z[U];
      int dst[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        dst[u] = r0 + min(e0 + u * nt, tot - 1);
        z[u] = cvt<C>(a.t[dst[u]]);
      }
      if (a.perm) {
#pragma unroll
        for (int u = 0; u < U; ++u) dst[u] = a.perm[dst[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e0 + u * nt < tot) st_out(&a.yout[dst[u]], cvt<typename P::O>(z[u] - x[e0 + u * nt]));
    } else {
      // unconditional clamped loads: all U in flight before the stores
      C z[U];
      int64_t g[U];
      int li[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int c, i;
        split_flat(min(e0 + u * nt, tot - 1), nr, nv, inv, c, i);
        g[u] = (int64_t)c * a.ldt + r0 + i;
        li[u] = c * xs + i;
        z[u] = cvt<C>(a.t[g[u]]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e0 + u * nt < tot) st_out(&a.t[g[u]], cvt<X>(z[u] - x[li[u]]));
    }
  }
}

// The C_l rows of TriArgs::ccopy that workgroup b writes to the caller's
// vector, by one wave (its stores left in flight)
template <class P>
__device__ __forceinline__ void copy_c_rows(const TriArgs<P>& a, int b, int lane) {
  using X = typename P::X;
  constexpr int U = 8;
  const int64_t lo = a.ccopy * b / a.nb, hi = a.ccopy * (b + 1) / a.nb;
  for (int64_t i0 = lo + lane; i0 < hi; i0 += (int64_t)kWave * U) {
    X v[U];
    int64_t dst[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      dst[u] = a.d + min(i0 + u * kWave, hi - 1);
      v[u] = a.t[dst[u]];
    }
    if (a.perm) {
#pragma unroll
      for (int u = 0; u < U; ++u) dst[u] = a.perm[dst[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * kWave < hi) st_out(&a.yout[dst[u]], cvt<typename P::O>(v[u]));
  }
}

// z1 of unit b under its E_l entries, ez[p] = x[row], from the records the
// producer staged in chunk buffer `buf` during the last chunk: eight
// records per thread in flight (clamped reads, padding p < 0 skipped)
template <class P>
__device__ __forceinline__ void file_e(const TriArgs<P>& a, int b, int buf, int nv, int tid, int nt,
                                       const uint8_t* bufs, const typename P::C* x, int xs) {
  using X = typename P::X;
  constexpr int U = 8;
  const int2* rec = reinterpret_cast<const int2*>(bufs + (size_t)buf * a.chunk_cap);
  const int nq = a.eunit[b + 1] - a.eunit[b];
  for (int q0 = tid; q0 < nq; q0 += nt * U) {
    int2 r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = rec[min(q0 + u * nt, nq - 1)];
    for (int c = 0; c < nv; ++c) {
      typename P::C v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = x[c * xs + r[u].y];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q0 + u * nt < nq && r[u].x >= 0) a.ez[(int64_t)c * a.ldez + r[u].x] = cvt<X>(v[u]);
    }
  }
}

// One workgroup per diagonal block (or group of blocks) and group of up to
// ncons vectors: waves 0 .. ncons - 1 sweep one vector each out of LDS,
// wave ncons copies the block's chunks.  All consumers sweep the same chunk
// between two barriers, so the factor entries cross HBM once for all of
// them.  Consumers without a vector (the launch's last group) only take
// part in the barriers.  MULTI false: one consumer and one vector per
// workgroup (vector blockIdx.y), with the register budget of two waves.
template <class P, int MS, int MODE, bool MULTI>
__global__ __launch_bounds__(MULTI ? kWave * (stream_max_cons(sizeof(typename P::C), MS) + 1)
                                   : 2 * kWave) void k_trisolve_streamed(
    TriArgs<P> a0) {
  using C = typename P::C;
  TriArgs<P> a = a0;
  const int ncons = MULTI ? a0.ncons : 1;
  const int g0 = (int)blockIdx.y * ncons;
  const int nv = MULTI ? min(ncons, a0.nvec - g0) : 1;
  a.t += (int64_t)g0 * a0.ldt;
  a.fy += (int64_t)g0 * a0.ldfy;
  if (MODE == TRI_DOWN && a.ez) a.ez += (int64_t)g0 * a0.ldez;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int nt = kWave * (ncons + 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // uniform: scalar branches
  const int lane = tid % kWave;
  const int r0 = a.blk_row[b];
  const int nr = a.blk_row[b + 1] - r0;
  // block vector of consumer c at byte c * x_bytes, the two buffers after
  C* x = reinterpret_cast<C*>(smem_raw);
  const int xs = a.x_bytes / (int)sizeof(C);
  uint8_t* bufs = smem_raw + (size_t)ncons * a.x_bytes;
  const int c0 = a.blk_chunk[b], c1 = a.blk_chunk[b + 1];
  // prologue unrolls within the register budget of the workgroup size
  constexpr int kU = 256 / (int)sizeof(C) < 32 ? 256 / (int)sizeof(C) : 32;
  // Down sweep of one vector whose block one round of loads covers: the
  // right-hand side's first loads (the permutation, or the values) go out
  // before the chunk descriptors' load, whose wait then covers them too --
  // one dependent round trip fewer before the sweep starts
  const bool pre = !MULTI && MODE == TRI_DOWN && nr <= nt * kU;
  int pidx[kU];
  C pval[kU];
  if (pre) {
    if (a.xin) {
#pragma unroll
      for (int u = 0; u < kU; ++u) pidx[u] = r0 + min(tid + u * nt, nr - 1);
      if (a.perm) {
#pragma unroll
        for (int u = 0; u < kU; ++u) pidx[u] = a.perm[pidx[u]];
      }
    } else {
#pragma unroll
      for (int u = 0; u < kU; ++u) pval[u] = cvt<C>(a.t[r0 + min(tid + u * nt, nr - 1)]);
    }
  }
  DescCache dc;
  if (c0 < c1) desc_fill<P>(a, c0, c1, lane, dc);
  const auto iters = [&](const ChunkDesc& cd) { return ((int)cd.n16 + kWave - 1) / kWave; };
  if (wave == ncons && c0 < c1) {
    const ChunkDesc cd = desc_get<P>(a, c0, c1, lane, dc);
    copy_chunk<P>(a, cd, bufs, lane, iters(cd));
  }
  if (pre) {
    if (a.xin) {
#pragma unroll
      for (int u = 0; u < kU; ++u) pval[u] = cvt<C>(a.xin[pidx[u]]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (tid + u * nt < nr) x[tid + u * nt] = pval[u];
  } else if (MODE == TRI_UP && a.frow) {
    rhs_from_f<P, MULTI ? 4 : 8>(a, b, nv, tid, nt, x, xs);
  } else {
    load_rhs<P, MODE, MULTI ? kU / 2 : kU>(a, r0, nr, nv, tid, nt, x, xs);
  }
  __syncthreads();
  for (int c = c0; c < c1; ++c) {
    const int k = c - c0;
    if (wave == ncons) {
      // the buffer of chunk c - 1 is free: fill it with chunk c + 1, then
      // wait until that has landed
      if (c + 1 < c1) {
        const ChunkDesc cd = desc_get<P>(a, c + 1, c1, lane, dc);
        copy_chunk<P>(a, cd, bufs + ((k + 1) % 2) * a.chunk_cap, lane, iters(cd));
      } else if (MODE == TRI_DOWN && a.erec) {
        // the last chunk: stage this unit's E_l records in the free buffer
        const int q0 = a.eunit[b], nq = a.eunit[b + 1] - q0;
        if (nq > 0)
          copy_to_lds(reinterpret_cast<const uint4*>(a.erec + 2 * (int64_t)q0), nq / 2,
                      bufs + ((k + 1) % 2) * a.chunk_cap, lane, (nq / 2 + kWave - 1) / kWave);
      }
      __builtin_amdgcn_s_waitcnt(GS_VMCNT_IMM(0));
      // the last chunk is being swept: the C_l rows meanwhile
      if constexpr (MODE == TRI_UP && !MULTI)
        if (c + 1 == c1 && a.ccopy > 0) copy_c_rows<P>(a, b, lane);
    } else {
      // Nothing of this wave is in flight here (its last chunk ended with a
      // full LDS wait), so this wait costs nothing; it tells the compiler
      // that the producer's LDS-DMA copies, which it cannot place on the
      // other wave, are not pending either -- otherwise it turns every LDS
      // wait of the sweep below into a full one.
      __builtin_amdgcn_s_waitcnt(0);
      const ChunkDesc cd = desc_get<P>(a, c, c1, lane, dc);
      if (wave < nv) {
        uint8_t* cur = bufs + (k % 2) * a.chunk_cap;
        // (the single-vector kernel keeps the constant base: every gather
        // address is then the stored offset itself)
        C* xv = MULTI ? x + wave * xs : x;
        // idle lanes store to the slot after the block's rows
        const int dummy = nr * (int)sizeof(C);
        if (cd.nst & 0x8000) {
          if (a.half_u) chunk_sweep<P, MS, true, true>(cur, cd, lane, xv, dummy);
          else chunk_sweep<P, MS, false, true>(cur, cd, lane, xv, dummy);
        } else {
          if (a.half_l) chunk_sweep<P, MS, true, false>(cur, cd, lane, xv, dummy);
          else chunk_sweep<P, MS, false, false>(cur, cd, lane, xv, dummy);
        }
      }
      // every read of the buffer done before the producer may refill it
      __builtin_amdgcn_s_waitcnt(GS_LGKM0_IMM);
    }
    // hand-over without a memory fence: copies of later chunks stay in flight
    __builtin_amdgcn_s_barrier();
  }
  if constexpr (MODE == TRI_UP && !MULTI)
    if (c0 >= c1 && wave == ncons && a.ccopy > 0) copy_c_rows<P>(a, b, lane);
  __syncthreads();
  if constexpr (MODE == TRI_DOWN)
    if (a.erec && c0 < c1) file_e<P>(a, b, (c1 - c0) % 2, nv, tid, nt, bufs, x, xs);
  store_result<P, MODE>(a, r0, nr, nv, tid, nt, x, xs);
}

template <class P, int MS, int MODE, bool MULTI>
static void launch_stream_kern(const TriArgs<P>& a, int nc, hipStream_t st) {
  const size_t lds = stream_lds_bytes(a.x_bytes, a.chunk_cap, nc);
  auto kern = k_trisolve_streamed<P, MS, MODE, MULTI>;
  static size_t attr_set = 65536;
  if (lds > attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    attr_set = lds;
  }
  TriArgs<P> b = a;
  b.ncons = nc;
  const unsigned groups = (unsigned)((std::max(a.nvec, 1) + nc - 1) / nc);
  hipLaunchKernelGGL(kern, dim3(a.nb, groups), dim3(kWave * (nc + 1)), lds, st, b);
}
template <class P, int MS, int MODE>
static void launch_stream_ms(const TriArgs<P>& a, hipStream_t st) {
  const int nc = std::max(1, std::min(a.ncons, stream_max_cons(sizeof(typename P::C), MS)));
  if (nc == 1) launch_stream_kern<P, MS, MODE, false>(a, 1, st);
  else launch_stream_kern<P, MS, MODE, true>(a, nc, st);
}

template <class P, int MODE>
static void launch_stream_mode(const TriArgs<P>& a, int maxslot, hipStream_t st) {
  // the layout was padded to stream_slots(maxslot) slots per stage
  const int ms = stream_slots(maxslot);
  if (ms == 4) launch_stream_ms<P, 4, MODE>(a, st);
  else if (ms == 8) launch_stream_ms<P, 8, MODE>(a, st);
  else if (ms == 10) launch_stream_ms<P, 10, MODE>(a, st);
  else if (ms == 12) launch_stream_ms<P, 12, MODE>(a, st);
  else launch_stream_ms<P, 16, MODE>(a, st);
}

// float64 values to a narrower storage type on the device, rounded as the
// host conversion rounds them (to float: nearest even; to bfloat16: the
// float value, then nearest even on its upper 16 bits)
template <class V> __device__ inline V store_from_double(double x);
template <> __device__ inline float store_from_double<float>(double x) { return (float)x; }
template <> __device__ inline bf16 store_from_double<bf16>(double x) {
  uint32_t u = __float_as_uint((float)x);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  bf16 b;
  b.u = (uint16_t)(u >> 16);
  return b;
}
template <class V>
__global__ __launch_bounds__(256) void k_store_from_double(const double* src, V* dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = store_from_double<V>(src[i]);
}
template <class V>
void launch_store_from_double(const double* src, V* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_store_from_double<V>, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
}
template void launch_store_from_double<float>(const double*, float*, int64_t, hipStream_t);
template void launch_store_from_double<bf16>(const double*, bf16*, int64_t, hipStream_t);

// fy = F_l y2 (most rows of B_l have no entry), so the up sweep's
// right-hand side is a plain load like the down sweep's.  Four rows per
// thread, 256 apart: four independent row-pointer -> entry -> y2 chains in
// flight per thread instead of one.
constexpr int kFyRows = 4;
template <class P>
__global__ __launch_bounds__(256) void k_fy(CsrDev<P> F, const typename P::X* y2,
                                            typename P::C* fy, int64_t d, int64_t ldy,
                                            int64_t ldfy) {
  using C = typename P::C;
  y2 += (int64_t)blockIdx.y * ldy;  // vector blockIdx.y of a batched launch
  fy += (int64_t)blockIdx.y * ldfy;
  const int64_t i0 = (int64_t)blockIdx.x * 256 * kFyRows + threadIdx.x;
  int rows[kFyRows];
#pragma unroll
  for (int q = 0; q < kFyRows; ++q) {
    const int64_t i = i0 + (int64_t)q * 256;
    rows[q] = i < d ? (int)i : -1;
  }
  C r[kFyRows];
  csr_rows<C, typename P::V, typename P::X, kFyRows, 2>(F.rp, F.ci, F.v, y2, rows, r);
#pragma unroll
  for (int q = 0; q < kFyRows; ++q)
    if (rows[q] >= 0) fy[rows[q]] = r[q];
}

template <class P>
void launch_trisolve_streamed(const TriArgs<P>& a, int mode, int maxslot, int max_block_rows,
                              hipStream_t st) {
  (void)max_block_rows;
  if (a.nb <= 0) return;
  if (mode == TRI_DOWN) {
    launch_stream_mode<P, TRI_DOWN>(a, maxslot, st);
  } else {
    if (!a.frow) {
      const dim3 gfy((unsigned)((a.d + 256 * kFyRows - 1) / (256 * kFyRows)), a.nvec);
      hipLaunchKernelGGL(k_fy<P>, gfy, dim3(256), 0, st, a.F, a.t + a.d, a.fy, a.d, a.ldt, a.ldfy);
    }
    launch_stream_mode<P, TRI_UP>(a, maxslot, st);
  }
}

// ======================================================================
// Interface step of one level: z2 = b2 - E_l z1 written in place, and the
// projection W^H z2 of the low-rank term: every workgroup leaves its
// partial sums, the last workgroup to finish adds them in workgroup order
// (deterministic) and applies H = (I - R)^{-1} - I, giving t' = H W^H z2.
// ======================================================================
constexpr int kIfThreads = 256;

// b2 of interface row i: t, or the caller's vector through the permutation
template <class P>
__device__ __forceinline__ typename P::C if_b2(const IfArgs<P>& a, int64_t i) {
  using C = typename P::C;
  using X = typename P::X;
  if (a.xin) {
    const int64_t g = a.d + i;
    return cvt<C>(cvt<X>(a.xin[a.perm ? a.perm[g] : g]));
  }
  return cvt<C>(a.t[a.d + i]);
}

// (E_l z1)[row] for R rows per thread: z1 gathered from t, or read in
// E_l's entry order from ez where the down sweep filed it (same products,
// same order of summation)
template <class P, int R>
__device__ __forceinline__ void e_rows(const IfArgs<P>& a, const int (&rows)[R],
                                       typename P::C (&r)[R]) {
  using C = typename P::C;
  using X = typename P::X;
  if (a.ez) csr_rows<C, typename P::V, X, R, 4, true>(a.E.rp, a.E.ci, a.E.v, a.ez, rows, r);
  else csr_rows<C, typename P::V, X, R, 4>(a.E.rp, a.E.ci, a.E.v, a.t, rows, r);
}

// z2 = b2 - E_l z1 of R rows per thread, written over t[d + row]; the rows
// of thread tid of workgroup g are g * 256 R + tid + q * 256
template <class P, int R>
__device__ __forceinline__ void if_z2(const IfArgs<P>& a, int64_t base,
                                      typename P::C (&z)[R]) {
  using C = typename P::C;
  using X = typename P::X;
  int rows[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t j = base + (int64_t)q * kIfThreads;
    rows[q] = j < a.s ? (int)j : -1;
  }
  C ez[R];
  e_rows<P, R>(a, rows, ez);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    z[q] = zero<C>();
    if (rows[q] >= 0) {
      const C acc = if_b2(a, rows[q]) - ez[q];
      a.t[a.d + rows[q]] = cvt<X>(acc);
      z[q] = acc;
    }
  }
}

template <class P, int R, int KG>
__global__ __launch_bounds__(kIfThreads) void k_interface(IfArgs<P> a0) {
  using C = typename P::C;
  using X = typename P::X;
  // vector blockIdx.y of a batched launch
  IfArgs<P> a = a0;
  a.t += (int64_t)blockIdx.y * a0.ldt;
  a.partial += (int64_t)blockIdx.y * a0.ldpart;
  if (a.ez) a.ez += (int64_t)blockIdx.y * a0.ldez;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* red = reinterpret_cast<C*>(smem_raw);  // 9 x kIfThreads (block_sum8)
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kIfThreads * R + tid;
  C z[R];
  if_z2<P, R>(a, base, z);
  if (a.k == 0) return;
  // W^H z2 for this workgroup's rows, KG columns at a time: the loads of all
  // KG columns are in flight together (unconditional, at clamped indices:
  // rows past s carry z = 0, columns past k are never written), then the KG
  // sums go over the workgroup 8 at a time, in fixed order, through LDS
  for (int c0 = 0; c0 < a.k; c0 += KG) {
    C pr[KG];
#pragma unroll
    for (int u = 0; u < KG; ++u) pr[u] = zero<C>();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t j = min(base + (int64_t)q * kIfThreads, a.s - 1);
#pragma unroll
      for (int u = 0; u < KG; ++u) {
        const int64_t cu = min(c0 + u, a.k - 1);
        pr[u] += conj(cvt<C>(a.W[j + cu * a.s])) * z[q];
      }
    }
#pragma unroll
    for (int u0 = 0; u0 < KG; u0 += 8) {
      if (c0 + u0 < a.k) {
        C p8[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) p8[v] = pr[u0 + v];
        const C sm = block_sum8(p8, red, tid);
        if (tid < 8 && c0 + u0 + tid < a.k)
          a.partial[(int64_t)blockIdx.x * a.k + c0 + u0 + tid] = sm;
      }
    }
  }
}

// t' = H (sum over workgroups of the partials), one workgroup of 1024
// threads: T = 1024 / k threads per column sum the partials of workgroups
// g, g+T, ... (coalesced: consecutive threads read consecutive columns, in
// batches of 8 loads), the T group sums are added in order in LDS; then
// thread (r, q) forms the part of row r of H t over columns q, q+T, ...
// (its first kFinishH entries of H fetched before the partials) and the
// parts are added in order.  Deterministic; no atomics.
constexpr int kFinishThreads = 1024;
constexpr int kFinishH = 4;

// v[0] + v[ld] + ... + v[(n - 1) ld] from LDS, added in that order, with
// eight reads in flight at a time (a loop of single reads waits out the
// LDS latency at every step)
template <class C>
__device__ __forceinline__ C lds_sum_ordered(const C* v, int ld, int n) {
  C t = zero<C>();
  int q = 0;
  for (; q + 8 <= n; q += 8) {
    C r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = v[(q + u) * ld];
#pragma unroll
    for (int u = 0; u < 8; ++u) t += r[u];
  }
  for (; q < n; ++q) t += v[q * ld];
  return t;
}

// sum of partial[b * rs + c * cs] over b = g, g + T, ... < nb, in that
// order, NL loads in flight at a time (clamped to the last row)
template <class C, int NL>
__device__ __forceinline__ C finish_part_sum(const C* partial, int nb, int64_t rs, int64_t cs,
                                             int T, int c, int g) {
  C s = zero<C>();
  for (int b = g; b < nb; b += NL * T) {
    C v[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) v[u] = partial[(int64_t)min(b + u * T, nb - 1) * rs + c * cs];
#pragma unroll
    for (int u = 0; u < NL; ++u) s = sel(b + u * T < nb, s + v[u], s);
  }
  return s;
}

// cld > 0: the partials are column-major, partial[c * cld + b] (as
// k_multidot leaves them), else partial[b * k + c].
template <class P>
__global__ __launch_bounds__(kFinishThreads) void k_project_finish(const typename P::C* partial,
                                                                   int nb, int k,
                                                                   const typename P::C* H,
                                                                   typename P::C* tprime,
                                                                   int64_t ldpart, int64_t cld) {
  using C = typename P::C;
  partial += (int64_t)blockIdx.y * ldpart;  // vector blockIdx.y of a batched launch
  tprime += (int64_t)blockIdx.y * k;
  __shared__ C red[kFinishThreads];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tv = reinterpret_cast<C*>(smem_raw);  // k
  const int tid = threadIdx.x;
  const int T = kFinishThreads / k;
  const int c = tid % k, g = tid / k;
  C h0[kFinishH];
#pragma unroll
  for (int u = 0; u < kFinishH; ++u) h0[u] = H[c + (int64_t)min(g + u * T, k - 1) * k];
  // (batches of 8: at level 0, k = 33, 636 partials, 24 or 32 loads in
  // flight per thread, mostly clamped repeats, measured no faster or
  // 1.3 us slower -- one CU's load pipe, not the round trips, bounds it)
  C s = zero<C>();
  if (g < T)
    s = cld > 0 ? finish_part_sum<C, 8>(partial, nb, 1, cld, T, c, g)
                : finish_part_sum<C, 8>(partial, nb, k, 1, T, c, g);
  red[tid] = s;
  __syncthreads();
  if (tid < k) tv[tid] = lds_sum_ordered<C>(red + tid, k, T);
  __syncthreads();
  s = zero<C>();
  if (g < T) {
#pragma unroll
    for (int u = 0; u < kFinishH; ++u) {
      const int cc = g + u * T;
      s = sel(cc < k, s + h0[u] * tv[min(cc, k - 1)], s);
    }
    for (int cc = g + kFinishH * T; cc < k; cc += 8 * T) {
      C h[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) h[u] = H[c + (int64_t)min(cc + u * T, k - 1) * k];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = sel(cc + u * T < k, s + h[u] * tv[min(cc + u * T, k - 1)], s);
    }
  }
  __syncthreads();
  red[tid] = s;
  __syncthreads();
  if (tid < k) tprime[tid] = lds_sum_ordered<C>(red + tid, k, T);
}

// rows per thread of the interface kernel: 2 when that still leaves two
// workgroups per CU and the column batch fits the registers of a resident
// workgroup (real types, k <= 40), else 1
template <class P>
static int interface_rows(int64_t s, int k) {
  using C = typename P::C;
  // (measured at level 0, k = 33: two rows 28 us, one row 31 us)
  return sizeof(C) < 16 && k <= 40 && s >= (int64_t)kIfThreads * 2 * 512 ? 2 : 1;
}

// upper bound of the workgroups launch_interface uses for s interface rows
// (the size of `partial` is this times k)
template <class P>
int interface_blocks(int64_t s) {
  return (int)((s + kIfThreads - 1) / kIfThreads);
}

template <class T>
__global__ __launch_bounds__(256) void k_multidot(const T* V, int64_t ld, int ncol, const T* w,
                                                  int64_t n, T* partial);
constexpr int kDotChunk = 8;     // columns per workgroup row of the grid
constexpr int kDotBlocks = 256;  // workgroups along the rows

// Ranks above two column batches (40 columns for float64, 16 for
// complex128; forms where W_l, z2 and the sums share one type): the E
// product alone first (k_interface with k = 0), then
// W^H z2 as a column-chunked multidot that streams W_l once over the whole
// chip, and the finish on its column-major partials.  One launch and one z2
// round trip more than the fused step, but no serial batches of block sums
// per workgroup (measured at 128^3, level 0: k = 256 212 -> 181 us, k = 129
// 113 -> 96 us; k = 65 even, level 1 at k = 64 1.7 us slower; complex128,
// k = 65: 97.9 -> 91.6 us).
template <class C> constexpr int if_fused_max_k() { return sizeof(C) == 16 ? 32 : 80; }
template <class P>
static bool interface_by_multidot(const IfArgs<P>& a, int R, hipStream_t st) {
  using C = typename P::C;
  if constexpr (!std::is_same<typename P::V, C>::value || !std::is_same<typename P::X, C>::value) {
    (void)a, (void)R, (void)st;
    return false;
  } else {
    if (a.k <= if_fused_max_k<C>()) return false;
    IfArgs<P> e = a;
    e.k = 0;
    const int nblk = (int)((a.s + (int64_t)kIfThreads * R - 1) / ((int64_t)kIfThreads * R));
    const size_t lds = (size_t)9 * kRedThreads * sizeof(C);
    if (R == 2)
      hipLaunchKernelGGL((k_interface<P, 2, 16>), dim3(nblk, a.nvec), dim3(kIfThreads), lds, st, e);
    else
      hipLaunchKernelGGL((k_interface<P, 1, 16>), dim3(nblk, a.nvec), dim3(kIfThreads), lds, st, e);
    const int nbm = (int)std::min<int64_t>(kDotBlocks, (a.s + 255) / 256);
    const dim3 grid(nbm, (a.k + kDotChunk - 1) / kDotChunk);
    for (int j = 0; j < a.nvec; ++j) {
      const C* z2 = a.t + (int64_t)j * a.ldt + a.d;
      C* part = a.partial + (int64_t)j * a.ldpart;
      hipLaunchKernelGGL(k_multidot<C>, grid, dim3(256), 0, st, a.W, a.s, a.k, z2, a.s, part);
      hipLaunchKernelGGL(k_project_finish<P>, dim3(1, 1), dim3(kFinishThreads),
                         (size_t)a.k * sizeof(C), st, part, nbm, a.k, a.H,
                         a.tprime + (int64_t)j * a.k, (int64_t)0, (int64_t)nbm);
    }
    return true;
  }
}

template <class P>
void launch_interface(const IfArgs<P>& a, hipStream_t st) {
  if (a.s <= 0) return;
  using C = typename P::C;
  const int R = interface_rows<P>(a.s, a.k);
  if (interface_by_multidot<P>(a, R, st)) return;
  const int nblk = (int)((a.s + (int64_t)kIfThreads * R - 1) / ((int64_t)kIfThreads * R));
  const size_t lds = (size_t)9 * kRedThreads * sizeof(C);
  // columns per load batch: all of k when it is small, else batches sized so
  // that the registers still allow every workgroup to be resident at once
#define GS_IF_LAUNCH(R_, KG) \
  hipLaunchKernelGGL((k_interface<P, R_, KG>), dim3(nblk, a.nvec), dim3(kIfThreads), lds, st, a)
  if constexpr (sizeof(C) == 16) {
    GS_IF_LAUNCH(1, 16);
  } else {
    if (R == 2 && a.k <= 16) GS_IF_LAUNCH(2, 16);
    else if (R == 2) GS_IF_LAUNCH(2, 40);
    else if (a.k <= 16) GS_IF_LAUNCH(1, 16);
    else GS_IF_LAUNCH(1, 40);
  }
#undef GS_IF_LAUNCH
  if (a.k > 0)
    hipLaunchKernelGGL(k_project_finish<P>, dim3(1, a.nvec), dim3(kFinishThreads),
                       (size_t)a.k * sizeof(C), st, a.partial, nblk, a.k, a.H, a.tprime, a.ldpart,
                       (int64_t)0);
}

// The whole interface step of a small level in one workgroup (s <= 4096,
// k <= 64): z2 = b2 - E_l z1, t = W^H z2, t' = H t and z2 + W t' written
// back, with z2 kept in LDS; one launch instead of three, for levels where
// launch latency, not bandwidth, is the cost.  Sums in fixed order.
// WL: W_l (s x k, at most kSmallW values per thread) and H_l are copied to
// LDS, their loads issued before the E-product's, so the step costs the
// E-product's dependent loads and not three more rounds of W and H loads.
constexpr int kSmallThreads = 1024;
constexpr int kSmallW = 16;
template <class P, bool WL>
__global__ __launch_bounds__(kSmallThreads) void k_interface_small(IfArgs<P> a0) {
  using C = typename P::C;
  using X = typename P::X;
  using V = typename P::V;
  using D = typename P::D;
  IfArgs<P> a = a0;  // vector blockIdx.y of a batched launch
  a.t += (int64_t)blockIdx.y * a0.ldt;
  if (a.ez) a.ez += (int64_t)blockIdx.y * a0.ldez;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = (int)a.s, k = a.k, tid = threadIdx.x;
  C* zs = reinterpret_cast<C*>(smem_raw);  // s
  C* red = zs + s;                          // kSmallThreads
  C* tv = red + kSmallThreads;              // k: W^H z2
  C* tp = tv + 64;                          // k: H W^H z2
  C* hs = tp + 64;                          // WL: H (k x k)
  V* ws = reinterpret_cast<V*>(hs + (WL ? k * k : 0));  // WL: W (s x k)
  X* tc = a.t + a.d;
  const int sk = s * k, kk = k * k;
  V wr[WL ? kSmallW : 1];
  C hr[WL ? 4 : 1];
  D dr[WL ? 4 : 1];
  if (WL && k > 0) {
#pragma unroll
    for (int m = 0; m < kSmallW; ++m) wr[m] = a.W[min(tid + m * kSmallThreads, sk - 1)];
#pragma unroll
    for (int m = 0; m < 4; ++m) hr[m] = a.H[min(tid + m * kSmallThreads, kk - 1)];
  }
  if (WL && a.last_dinv) {
#pragma unroll
    for (int m = 0; m < 4; ++m) dr[m] = a.last_dinv[min(tid + m * kSmallThreads, s - 1)];
  }
  for (int i = tid; i < s; i += kSmallThreads) {
    const int rows[1] = {i};
    C ez[1];
    e_rows<P, 1>(a, rows, ez);
    zs[i] = if_b2(a, i) - ez[0];
  }
  if (WL && k > 0) {
#pragma unroll
    for (int m = 0; m < kSmallW; ++m)
      if (tid + m * kSmallThreads < sk) ws[tid + m * kSmallThreads] = wr[m];
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (tid + m * kSmallThreads < kk) hs[tid + m * kSmallThreads] = hr[m];
  }
  __syncthreads();
  const V* Wv = WL ? ws : a.W;
  const C* Hv = WL ? hs : a.H;
  // the C-part's final value: w, or the diagonal last level's solve of it
  // (as that level's sweep computes it: (w - 0) * 1/u_ii); m: i's index
  // among the thread's rows
  const auto put = [&](int i, int m, const C& w) {
    if (a.last_dinv) {
      const D dv = WL ? dr[m] : a.last_dinv[i];
      tc[i] = cvt<X>(cvt<C>(cvt<X>(w)) * cvt<C>(dv));
    } else {
      tc[i] = cvt<X>(w);
    }
  };
  // s <= 4096: at most four rows per thread
  if (k == 0) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (tid + m * kSmallThreads < s) put(tid + m * kSmallThreads, m, zs[tid + m * kSmallThreads]);
    return;
  }
  // T threads per column, thread (c, g) sums rows g, g + T, ...
  const int T = kSmallThreads / k;
  const int c = tid % k, g = tid / k;
  C acc = zero<C>();
  if (g < T) {
#pragma unroll 8
    for (int i = g; i < s; i += T) acc += conj(cvt<C>(Wv[i + (int64_t)c * s])) * zs[i];
  }
  red[tid] = acc;
  __syncthreads();
  if (tid < k) {
    C t = zero<C>();
    for (int q = 0; q < T; ++q) t += red[q * k + tid];
    tv[tid] = t;
  }
  __syncthreads();
  if (tid < k) {
    C t = zero<C>();
    for (int q = 0; q < k; ++q) t += Hv[tid + (int64_t)q * k] * tv[q];
    tp[tid] = t;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int i = tid + m * kSmallThreads;
    if (i >= s) break;
    C w = zs[i];
#pragma unroll 8
    for (int q = 0; q < k; ++q) w += cvt<C>(Wv[i + (int64_t)q * s]) * tp[q];
    put(i, m, w);
  }
}

template <class P, bool WL>
static void launch_small_wl(const IfArgs<P>& a, size_t lds, hipStream_t st) {
  static size_t attr_set = 65536;
  if (lds > attr_set) {
    (void)hipFuncSetAttribute((const void*)k_interface_small<P, WL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr_set = lds;
  }
  hipLaunchKernelGGL((k_interface_small<P, WL>), dim3(1, a.nvec), dim3(kSmallThreads), lds, st, a);
}

template <class P>
bool launch_interface_small(const IfArgs<P>& a, hipStream_t st) {
  using C = typename P::C;
  using V = typename P::V;
  if (a.s <= 0 || a.s > 4096 || a.k > 64) return false;
  const size_t base = ((size_t)a.s + kSmallThreads + 128) * sizeof(C);
  const size_t wl = base + (size_t)a.k * a.k * sizeof(C) + (size_t)a.s * a.k * sizeof(V) + 16;
  // (real forms only: complex W values would not stay in registers)
  if constexpr (sizeof(V) <= 8) {
    if (a.stage_w && a.k > 0 && a.s * a.k <= (int64_t)kSmallW * kSmallThreads &&
        a.k * a.k <= 4 * kSmallThreads && wl <= (size_t)a.max_lds) {
      launch_small_wl<P, true>(a, wl, st);
      return true;
    }
  }
  launch_small_wl<P, false>(a, base, st);
  return true;
}

// t_C += W t'
template <class P>
__global__ __launch_bounds__(256) void k_lowrank_update(typename P::X* tc, int64_t s, int k,
                                                        const typename P::V* W,
                                                        const typename P::C* tprime,
                                                        int64_t ldt) {
  using C = typename P::C;
  using X = typename P::X;
  tc += (int64_t)blockIdx.y * ldt;  // vector blockIdx.y of a batched launch
  tprime += (int64_t)blockIdx.y * k;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* tp = reinterpret_cast<C*>(smem_raw);
  for (int c = threadIdx.x; c < k; c += blockDim.x) tp[c] = tprime[c];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= s) return;
  C acc = cvt<C>(tc[j]);
  for (int c = 0; c < k; ++c) acc += cvt<C>(W[j + (int64_t)c * s]) * tp[c];
  tc[j] = cvt<X>(acc);
}

template <class P>
void launch_lowrank_update(typename P::X* tc, int64_t s, int k, const typename P::V* W,
                           const typename P::C* tprime, hipStream_t st, int nvec, int64_t ldt) {
  if (s <= 0 || k <= 0 || nvec <= 0) return;
  const int nblk = (int)((s + 255) / 256);
  hipLaunchKernelGGL(k_lowrank_update<P>, dim3(nblk, nvec), dim3(256),
                     (size_t)k * sizeof(typename P::C), st, tc, s, k, W, tprime, ldt);
}

// ---------------------------------------------------------------- perm
template <class P>
__global__ void k_gather(const typename P::O* x, const int32_t* perm, typename P::X* t,
                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t src = perm ? perm[i] : i;
  t[i] = cvt<typename P::X>(x[src]);
}
template <class P>
__global__ void k_scatter(const typename P::X* t, const int32_t* perm, typename P::O* y,
                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t dst = perm ? perm[i] : i;
  y[dst] = cvt<typename P::O>(t[i]);
}
template <class P>
void launch_gather(const typename P::O* x, const int32_t* perm, typename P::X* t, int64_t n,
                   hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather<P>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, perm,
                     t, n);
}
template <class P>
void launch_scatter(const typename P::X* t, const int32_t* perm, typename P::O* y, int64_t n,
                    hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter<P>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, t,
                     perm, y, n);
}

// ======================================================================
// float64 / complex128 vector kernels (FGMRES, Arnoldi)
// ======================================================================
// One row of a CSR product, y_i = acc0 + sum_p v_p x[ci_p] in stored order
// (acc0 = 0, or -b_i negated below for the residual).  Up to kRowU entries of
// the row are loaded at once (columns and values in one round trip, then the
// x gathers in a second), longer rows continue in further rounds: three
// dependent round trips per thread for a stencil row instead of two per
// entry.  Entries past the row end are loaded at its last index and add an
// exact zero.
constexpr int kRowU = 8;
template <class T>
__device__ __forceinline__ T csr_row_dot(const int32_t* rp, const int32_t* ci, const T* v,
                                         const T* x, int64_t i) {
  const int p0 = rp[i], p1 = rp[i + 1];
  T acc = zero<T>();
  for (int pb = p0; pb < p1; pb += kRowU) {
    int c[kRowU];
    T w[kRowU];
#pragma unroll
    for (int u = 0; u < kRowU; ++u) {
      const int p = min(pb + u, p1 - 1);
      c[u] = ci[p];
      w[u] = v[p];
    }
    T xv[kRowU];
#pragma unroll
    for (int u = 0; u < kRowU; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < kRowU; ++u)
      if (pb + u < p1) acc += w[u] * xv[u];
  }
  return acc;
}

template <class T>
__global__ __launch_bounds__(256) void k_spmv(const int32_t* rp, const int32_t* ci, const T* v,
                                              const T* x, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = csr_row_dot(rp, ci, v, x, i);
}
template <class T>
void launch_spmv(const int32_t* rp, const int32_t* ci, const T* v, const T* x, T* y, int64_t n,
                 hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_spmv<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rp, ci, v,
                     x, y, n);
}

// y = b - A x, the row's products subtracted from b_i one by one in stored
// order (the operations of the plain loop)
template <class T>
__global__ __launch_bounds__(256) void k_residual(const int32_t* rp, const int32_t* ci,
                                                  const T* v, const T* x, const T* b, T* y,
                                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = rp[i], p1 = rp[i + 1];
  T acc = b[i];
  for (int pb = p0; pb < p1; pb += kRowU) {
    int c[kRowU];
    T w[kRowU];
#pragma unroll
    for (int u = 0; u < kRowU; ++u) {
      const int p = min(pb + u, p1 - 1);
      c[u] = ci[p];
      w[u] = v[p];
    }
    T xv[kRowU];
#pragma unroll
    for (int u = 0; u < kRowU; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < kRowU; ++u)
      if (pb + u < p1) acc -= w[u] * xv[u];
  }
  y[i] = acc;
}
template <class T>
void launch_residual(const int32_t* rp, const int32_t* ci, const T* v, const T* x, const T* b,
                     T* y, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_residual<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rp, ci,
                     v, x, b, y, n);
}

template <class T>
__global__ __launch_bounds__(256) void k_multidot(const T* V, int64_t ld, int ncol,
                                                  const T* w, int64_t n, T* partial) {
  __shared__ T red[9 * kRedThreads];
  const int c0 = blockIdx.y * kDotChunk;
  const int nc = min(kDotChunk, ncol - c0);
  T acc[kDotChunk];
#pragma unroll
  for (int c = 0; c < kDotChunk; ++c) acc[c] = zero<T>();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T wi = w[i];
#pragma unroll
    for (int c = 0; c < kDotChunk; ++c)
      if (c < nc) acc[c] += conj(V[i + (int64_t)(c0 + c) * ld]) * wi;
  }
  const T s = block_sum8(acc, red, threadIdx.x);
  if (threadIdx.x < nc) partial[(int64_t)(c0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
}
// h[c] = sum_b partial[c][b]: one workgroup per column, fixed-order tree
template <class T>
__global__ __launch_bounds__(256) void k_sum_partials(const T* partial, int nparts, int ncol,
                                                      T* h) {
  __shared__ T red[kRedThreads + 32];
  const int c = blockIdx.x;
  T s = threadIdx.x < nparts ? partial[(int64_t)c * nparts + threadIdx.x] : zero<T>();
  s = block_sum1(s, red, threadIdx.x);
  if (threadIdx.x == 0) h[c] = s;
}
template <class T>
void launch_multidot(const T* V, int64_t ld, int ncol, const T* w, int64_t n, T* partial, T* h,
                     hipStream_t st) {
  if (ncol <= 0) return;
  const int nb = (int)std::min<int64_t>(kDotBlocks, (n + 255) / 256);
  dim3 grid(nb, (ncol + kDotChunk - 1) / kDotChunk);
  hipLaunchKernelGGL(k_multidot<T>, grid, dim3(256), 0, st, V, ld, ncol, w, n, partial);
  hipLaunchKernelGGL(k_sum_partials<T>, dim3(ncol), dim3(256), 0, st, partial, nb, ncol, h);
}

template <class T>
__global__ void k_gemv_sub(const T* V, int64_t ld, int ncol, const T* h, T* w, int64_t n,
                           T* hacc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* hs = reinterpret_cast<T*>(smem_raw);
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) hs[c] = h[c];
  __syncthreads();
  if (hacc && blockIdx.x == 0)
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) hacc[c] += hs[c];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T acc = w[i];
  for (int c = 0; c < ncol; ++c) acc -= V[i + (int64_t)c * ld] * hs[c];
  w[i] = acc;
}
template <class T>
void launch_gemv_sub(const T* V, int64_t ld, int ncol, const T* h, T* w, int64_t n, T* hacc,
                     hipStream_t st) {
  if (ncol <= 0) return;
  hipLaunchKernelGGL(k_gemv_sub<T>, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     (size_t)ncol * sizeof(T), st, V, ld, ncol, h, w, n, hacc);
}

template <class T>
__global__ __launch_bounds__(256) void k_norm_part(const T* w, int64_t n, double* partial) {
  __shared__ double red[kRedThreads + 32];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += norm2(w[i]);
  acc = block_sum1(acc, red, threadIdx.x);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}
__global__ __launch_bounds__(256) void k_norm_final(const double* partial, int nparts,
                                                    double* out) {
  __shared__ double red[kRedThreads + 32];
  double s = threadIdx.x < nparts ? partial[threadIdx.x] : 0.0;
  s = block_sum1(s, red, threadIdx.x);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}
template <class T>
void launch_norm(const T* w, int64_t n, double* partial, double* out, hipStream_t st) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (n + 255) / 256));
  hipLaunchKernelGGL(k_norm_part<T>, dim3(nb), dim3(256), 0, st, w, n, partial);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, st, partial, nb, out);
}

template <class T>
__global__ void k_scale_inv(const T* x, const double* nrm, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = nrm[0];
  y[i] = s > 0.0 ? x[i] * (1.0 / s) : zero<T>();
}
template <class T>
void launch_scale_inv(const T* x, const double* nrm, T* y, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale_inv<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, nrm,
                     y, n);
}

// One Arnoldi step recorded on the device: the new Hessenberg column h
// (cnt entries) and the norms (nrm[0] = ||w|| after orthogonalisation,
// nrm[1] = before) go to Scol and nd; y = w / nrm[0], or zero with *flag
// set when nrm[0] <= 1e-12 nrm[1] (breakdown: the host then redoes the
// cycle step by step).
template <class T>
__global__ void k_arnoldi_step(const T* h, int cnt, const double* nrm, T* Scol, double* nd,
                               double* flag, const T* w, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double beta = nrm[0], wn = nrm[1];
  const bool ok = beta > 1e-12 * wn;
  if (blockIdx.x == 0) {
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) Scol[q] = h[q];
    if (threadIdx.x == 0) {
      nd[0] = beta;
      nd[1] = wn;
      if (!ok) flag[0] = 1.0;
    }
  }
  if (i >= n) return;
  y[i] = ok ? w[i] * (1.0 / beta) : zero<T>();
}
template <class T>
void launch_arnoldi_step(const T* h, int cnt, const double* nrm, T* Scol, double* nd, double* flag,
                         const T* w, T* y, int64_t n, hipStream_t st) {
  // at least one block: block 0 records h and the norms
  const int64_t nblk = n > 0 ? (n + 255) / 256 : 1;
  hipLaunchKernelGGL(k_arnoldi_step<T>, dim3((unsigned)nblk), dim3(256), 0, st, h, cnt, nrm, Scol,
                     nd, flag, w, y, n);
}

template <class T>
__global__ void k_gemv_add(const T* Z, int64_t ld, int ncol, const T* y, T* x, int64_t n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* ys = reinterpret_cast<T*>(smem_raw);
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) ys[c] = y[c];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T acc = x[i];
  for (int c = 0; c < ncol; ++c) acc += Z[i + (int64_t)c * ld] * ys[c];
  x[i] = acc;
}
template <class T>
void launch_gemv_add(const T* Z, int64_t ld, int ncol, const T* y, T* x, int64_t n,
                     hipStream_t st) {
  if (ncol <= 0) return;
  hipLaunchKernelGGL(k_gemv_add<T>, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     (size_t)ncol * sizeof(T), st, Z, ld, ncol, y, x, n);
}

// Y (n x k) = V (n x m) G (m x k); G staged through LDS in column chunks
template <class T>
__global__ void k_gemm_small(const T* V, int64_t ld, int m, const T* G, int k, T* Y,
                             int64_t ldy, int64_t n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* gs = reinterpret_cast<T*>(smem_raw);
  const int c = blockIdx.y;
  for (int i = threadIdx.x; i < m; i += blockDim.x) gs[i] = G[(int64_t)c * m + i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  T acc = zero<T>();
  for (int i = 0; i < m; ++i) acc += V[r + (int64_t)i * ld] * gs[i];
  Y[r + (int64_t)c * ldy] = acc;
}
template <class T>
void launch_gemm_small(const T* V, int64_t ld, int m, const T* G, int k, T* Y, int64_t ldy,
                       int64_t n, hipStream_t st) {
  if (k <= 0 || m <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256), k);
  hipLaunchKernelGGL(k_gemm_small<T>, grid, dim3(256), (size_t)m * sizeof(T), st, V, ld, m, G, k,
                     Y, ldy, n);
}

template <class T>
__global__ void k_fill(T* x, T v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
template <class T>
void launch_fill(T* x, T v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, v, n);
}
template <class T>
__global__ void k_copy(const T* x, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}
template <class T>
void launch_copy(const T* x, T* y, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, n);
}

template <class T>
__global__ void k_permute(const T* x, const int32_t* perm, T* y, int64_t n, int scatter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (scatter) y[perm[i]] = x[i];
  else y[i] = x[perm[i]];
}
template <class T>
void launch_permute(const T* x, const int32_t* perm, T* y, int64_t n, bool scatter,
                    hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_permute<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, perm,
                     y, n, scatter ? 1 : 0);
}

template <class T>
__global__ void k_rows_to_cols(const float* Y, int64_t s, int k, int ldy, T* V, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s * k) return;
  const int64_t r = i / k, c = i % k;
  V[r + c * ld] = cvt_rc<T>(Y[r * ldy + c]);
}
template <class T>
void launch_rows_to_cols(const float* Y, int64_t s, int k, int ldy, T* V, int64_t ld,
                         hipStream_t st) {
  if (s * k <= 0) return;
  hipLaunchKernelGGL(k_rows_to_cols<T>, dim3((unsigned)((s * k + 255) / 256)), dim3(256), 0, st,
                     Y, s, k, ldy, V, ld);
}
template <class T>
__global__ void k_sub(const T* a, const T* b, T* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}
template <class T>
void launch_sub(const T* a, const T* b, T* out, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sub<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, out, n);
}

// ---------------------------------------------------------------- instances
// ======================================================================
// Small least-squares problem of the inner GMRES at the root level: with
// the Arnoldi relation S Z_m = V_{m+1} Hbar_m, c minimises
// ||beta e_1 - Hbar_m c||.  Hbar's column j holds h[j (m+1) + i], i <= j,
// and the real subdiagonal sub[j+1]; a step whose new direction vanished
// (sub[j+1] <= 1e-12 wn[j+1], wn = norm before orthogonalisation) ends the
// space there and later coefficients are zero.  Plane rotations with a real
// cosine reduce Hbar to triangular form; one thread, m <= kInnerMax.
// ======================================================================
__device__ inline double absv(double a) { return fabs(a); }
__device__ inline double absv(dcplx a) { return sqrt(norm2(a)); }
__device__ inline double scal(double a, double s) { return a * s; }
__device__ inline dcplx scal(dcplx a, double s) { return a * s; }
__device__ inline double divv(double a, double b) { return a / b; }
__device__ inline dcplx divv(dcplx a, dcplx b) { return scal(a * conj(b), 1.0 / norm2(b)); }
template <class T> __device__ inline T from_real(double a);
template <> __device__ inline double from_real<double>(double a) { return a; }
template <> __device__ inline dcplx from_real<dcplx>(double a) { return mk(a, 0.0); }

template <class T>
__global__ void k_inner_lsq(const T* h, const double* sub, const double* wn, const double* beta,
                            int m, T* c) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  T R[kInnerMax * kInnerMax];
  T g[kInnerMax + 1];
  double cs[kInnerMax];
  T sn[kInnerMax];
  for (int j = 0; j < m; ++j) c[j] = from_real<T>(0.0);
  if (!(beta[0] > 0)) return;
  int me = m;
  for (int j = 0; j < m; ++j)
    if (!(sub[j + 1] > 1e-12 * wn[j + 1])) { me = j + 1; break; }
  for (int i = 0; i <= m; ++i) g[i] = from_real<T>(0.0);
  g[0] = from_real<T>(beta[0]);
  for (int j = 0; j < me; ++j) {
    T col[kInnerMax + 1];
    for (int i = 0; i <= j; ++i) col[i] = h[(size_t)j * (m + 1) + i];
    col[j + 1] = from_real<T>(sub[j + 1]);
    for (int i = 0; i < j; ++i) {
      const T x = col[i], y = col[i + 1];
      col[i] = scal(x, cs[i]) + sn[i] * y;
      col[i + 1] = scal(y, cs[i]) - conj(sn[i]) * x;
    }
    const double aa = absv(col[j]), bb = sub[j + 1];
    const double r = sqrt(aa * aa + bb * bb);
    if (r == 0) {
      cs[j] = 1.0;
      sn[j] = from_real<T>(0.0);
    } else if (aa == 0) {
      cs[j] = 0.0;
      sn[j] = from_real<T>(1.0);
    } else {
      cs[j] = aa / r;
      sn[j] = scal(col[j], bb / (aa * r));  // (a/|a|) conj(b) / r with b real
    }
    const T x = col[j];
    col[j] = scal(x, cs[j]) + scal(sn[j], bb);
    for (int i = 0; i <= j; ++i) R[j * kInnerMax + i] = col[i];
    const T gx = g[j], gy = g[j + 1];
    g[j] = scal(gx, cs[j]) + sn[j] * gy;
    g[j + 1] = scal(gy, cs[j]) - conj(sn[j]) * gx;
  }
  for (int j = me - 1; j >= 0; --j) {
    T acc = g[j];
    for (int i = j + 1; i < me; ++i) acc -= R[i * kInnerMax + j] * c[i];
    const T d = R[j * kInnerMax + j];
    c[j] = absv(d) > 0 ? divv(acc, d) : from_real<T>(0.0);
  }
}

template <class T>
void launch_inner_lsq(const T* h, const double* sub, const double* wn, const double* beta, int m,
                      T* c, hipStream_t st) {
  hipLaunchKernelGGL(k_inner_lsq<T>, dim3(1), dim3(64), 0, st, h, sub, wn, beta, m, c);
}

#define GS_PREC_INSTANCES(P)                                                                   \
  template void launch_trisolve<P>(const TriArgs<P>&, int, int, int, hipStream_t);             \
  template void launch_trisolve_streamed<P>(const TriArgs<P>&, int, int, int, hipStream_t);    \
  template void launch_interface<P>(const IfArgs<P>&, hipStream_t);                            \
  template bool launch_interface_small<P>(const IfArgs<P>&, hipStream_t);                            \
  template int interface_blocks<P>(int64_t);                                                   \
  template void launch_lowrank_update<P>(P::X*, int64_t, int, const P::V*, const P::C*,        \
                                         hipStream_t, int, int64_t);                           \
  template void launch_gather<P>(const P::O*, const int32_t*, P::X*, int64_t, hipStream_t);    \
  template void launch_scatter<P>(const P::X*, const int32_t*, P::O*, int64_t, hipStream_t);
GS_PREC_INSTANCES(PF64)
GS_PREC_INSTANCES(PC128)
GS_PREC_INSTANCES(PF32)
GS_PREC_INSTANCES(PBF16)

#define GS_VEC_INSTANCES(T)                                                                    \
  template void launch_spmv<T>(const int32_t*, const int32_t*, const T*, const T*, T*,         \
                               int64_t, hipStream_t);                                          \
  template void launch_residual<T>(const int32_t*, const int32_t*, const T*, const T*,         \
                                   const T*, T*, int64_t, hipStream_t);                        \
  template void launch_multidot<T>(const T*, int64_t, int, const T*, int64_t, T*, T*,          \
                                   hipStream_t);                                               \
  template void launch_gemv_sub<T>(const T*, int64_t, int, const T*, T*, int64_t, T*,          \
                                   hipStream_t);                                               \
  template void launch_norm<T>(const T*, int64_t, double*, double*, hipStream_t);              \
  template void launch_scale_inv<T>(const T*, const double*, T*, int64_t, hipStream_t);        \
  template void launch_arnoldi_step<T>(const T*, int, const double*, T*, double*, double*,     \
                                       const T*, T*, int64_t, hipStream_t);                    \
  template void launch_gemv_add<T>(const T*, int64_t, int, const T*, T*, int64_t,              \
                                   hipStream_t);                                               \
  template void launch_gemm_small<T>(const T*, int64_t, int, const T*, int, T*, int64_t,       \
                                     int64_t, hipStream_t);                                    \
  template void launch_fill<T>(T*, T, int64_t, hipStream_t);                                   \
  template void launch_copy<T>(const T*, T*, int64_t, hipStream_t);                          \
  template void launch_permute<T>(const T*, const int32_t*, T*, int64_t, bool, hipStream_t);   \
  template void launch_rows_to_cols<T>(const float*, int64_t, int, int, T*, int64_t,         \
                                       hipStream_t);                                          \
  template void launch_sub<T>(const T*, const T*, T*, int64_t, hipStream_t);                  \
  template void launch_inner_lsq<T>(const T*, const double*, const double*, const double*, int, \
                                    T*, hipStream_t);
GS_VEC_INSTANCES(double)
GS_VEC_INSTANCES(dcplx)
template void launch_fill<float>(float*, float, int64_t, hipStream_t);

}  // namespace gs
