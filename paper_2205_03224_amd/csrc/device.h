// Device-side types, kernel argument blocks and launcher declarations of
// libgemslr.  Shared by the kernels (kernels.hip) and the host orchestration
// (gemslr.hip); not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

// ------------------------------------------------------------ scalar types
struct dcplx {
  double x, y;
};
__host__ __device__ inline dcplx mk(double a, double b) { dcplx r; r.x = a; r.y = b; return r; }
__host__ __device__ inline dcplx operator+(dcplx a, dcplx b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline dcplx operator-(dcplx a, dcplx b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline dcplx operator-(dcplx a) { return mk(-a.x, -a.y); }
__host__ __device__ inline dcplx operator*(dcplx a, dcplx b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline dcplx operator*(dcplx a, double s) { return mk(a.x * s, a.y * s); }
__host__ __device__ inline dcplx& operator+=(dcplx& a, dcplx b) { a = a + b; return a; }
__host__ __device__ inline dcplx& operator-=(dcplx& a, dcplx b) { a = a - b; return a; }
__host__ __device__ inline dcplx& operator*=(dcplx& a, dcplx b) { a = a * b; return a; }
__host__ __device__ inline dcplx conj(dcplx a) { return mk(a.x, -a.y); }
__host__ __device__ inline double conj(double a) { return a; }
__host__ __device__ inline float conj(float a) { return a; }
__host__ __device__ inline double norm2(dcplx a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double norm2(double a) { return a * a; }
__host__ __device__ inline float norm2(float a) { return a * a; }

// bfloat16 storage (upper half of a float32, round-to-nearest-even on the
// host when packing)
struct bf16 {
  uint16_t u;
};

// conversions between storage, compute and vector types
__device__ inline double cvt_d(double a) { return a; }
__device__ inline double cvt_d(float a) { return (double)a; }
__device__ inline float cvt_f(float a) { return a; }
__device__ inline float cvt_f(double a) { return (float)a; }
__device__ inline float cvt_f(bf16 a) { return __uint_as_float(((uint32_t)a.u) << 16); }

template <class To, class From> struct Cvt;
template <> struct Cvt<double, double> { __device__ static double f(double a) { return a; } };
template <> struct Cvt<float, float> { __device__ static float f(float a) { return a; } };
template <> struct Cvt<float, double> { __device__ static float f(double a) { return (float)a; } };
template <> struct Cvt<double, float> { __device__ static double f(float a) { return (double)a; } };
template <> struct Cvt<float, bf16> { __device__ static float f(bf16 a) { return __uint_as_float(((uint32_t)a.u) << 16); } };
template <> struct Cvt<dcplx, dcplx> { __device__ static dcplx f(dcplx a) { return a; } };
template <class To, class From> __device__ inline To cvt(From a) { return Cvt<To, From>::f(a); }

// Precision traits: V = stored factor/E/F/W value, C = compute, X = element
// of the working vector, D = stored inverse diagonal, O = element of the
// user-facing vectors (float64 or complex128).
struct PF64  { using V = double; using C = double; using X = double; using D = double; using O = double; };
struct PC128 { using V = dcplx;  using C = dcplx;  using X = dcplx;  using D = dcplx;  using O = dcplx; };
struct PF32  { using V = float;  using C = float;  using X = float;  using D = float;  using O = double; };
struct PBF16 { using V = bf16;   using C = float;  using X = float;  using D = float;  using O = double; };

// ------------------------------------------------------------ layouts
// One triangle (L or U) of one level, all diagonal blocks, in the
// level-scheduled "stage" layout: each block's rows are grouped by
// wavefront level, each level cut into stages of at most 64 rows; inside a
// stage rows are sorted by entry count (descending) and the entries are
// stored slot-major (the j-th entry of every row that has one, then the
// (j+1)-th ...), so the 64 lanes of a wave read consecutive addresses.
template <class P>
struct TriDev {
  const int32_t* blk_stage;  // nb+1: stage range of each block
  const int32_t* stage_row;  // nstages+1: row-slot offsets
  const int32_t* stage_ent;  // nstages+1: entry offsets
  const uint32_t* rowinfo;   // per row slot: block-local row | count << 16
  const typename P::D* dinv; // per row slot, U only: 1/u_ii
  const typename P::V* val;  // entries
  const uint16_t* col;       // block-local column of each entry
};

template <class P>
struct CsrDev {
  const int32_t* rp;
  const int32_t* ci;
  const typename P::V* v;
};

enum { TRI_DOWN = 0, TRI_UP = 1 };

// Streamed form of the same stages: each block's L stages, then its U
// stages, packed into chunks of whole stages, each chunk one contiguous,
// 16-byte aligned byte range:
//   values       rows x VS x V          (offset 0)
//   inverse diag rows x D               (U chunks only)
//   row info     (rows + 1) x uint32: LDS byte offset of the row in the block
//                vector (row * sizeof(C), 24 bits) | stage rows << 24
//                (the last word zero: reading past the last stage gives 0 rows)
//   columns      (rows + 1) x CS x uint16 (the last row all zero)
// Each row of the chunk (rows of consecutive stages follow each other) holds
// its MS slots contiguously (MS = stream_slots(level's longest row)): the
// row's entries, with the near ones (see near_slots) in the last slots of
// each lane's share, and zero values with column 0 in the slots left over.
// In half-row stages lanes l and l + 32 share row l, lane l taking slots
// 0 .. MS/2 - 1 and lane l + 32 the rest.  The row strides VS =
// MS + 1 values and CS column entries make the per-lane accesses of a wave
// free of LDS bank conflicts, and let every slot be an immediate offset from
// one address per stage.  Columns are stored as LDS byte offsets of the
// block-vector element (row * ColScale<C>), so a gather needs no index
// arithmetic.  Section offsets are in 16-byte units.  A stage's first row
// follows from the previous stage, so the consumer needs no stage table.
struct ChunkDesc {
  uint32_t off;      // byte offset of the chunk in the level's blob
  uint16_t n16;      // chunk size in 16-byte units
  uint16_t nst;      // stages in the chunk | 0x8000 for U chunks
  uint16_t nrows;    // rows in the chunk
  uint16_t dinv16, info16, col16;
};

// slot count of the streamed layout for a level whose longest row has
// `maxslot` off-diagonal entries (0: no streamed kernel for it)
__host__ __device__ constexpr int stream_slots(int maxslot) {
  return maxslot <= 4 ? 4 : maxslot <= 8 ? 8 : maxslot <= 10 ? 10 : maxslot <= 12 ? 12
         : maxslot <= 16 ? 16 : 0;
}
__host__ __device__ constexpr int stream_vstride(int ms) { return ms + 1; }
__host__ __device__ constexpr int stream_cstride(int ms) { return ms <= 4 ? 4 : ms <= 12 ? 12 : 20; }
// half-row stages: a row's slots ms/2 .. ms-1 start at this 16-bit
// position of its column row (the next 4-byte boundary)
__host__ __device__ constexpr int stream_half_coff(int ms) { return ((ms / 2) + 1) & ~1; }
// Near slots per lane: the last near_slots(ms, half) slots of each lane's
// share of a row hold the entries whose column was computed by the stage
// just before (plus, if the row has fewer such entries, any others).  The
// sweep gathers them after that stage's store; every other slot refers to a
// stage at least two back and is gathered a stage ahead.  The layout keeps
// at most this many near entries per lane (a stage that would hold more is
// split).
__host__ __device__ constexpr int near_slots(int ms, bool half) {
  return half ? (ms / 2 < 2 ? ms / 2 : 2) : (ms < 3 ? ms : 3);
}
// byte scale of the stored column: the element size, so the stored value is
// the element's LDS byte offset (16-bit: blocks of up to 65536 / sizeof(C)
// rows use the streamed layout)
template <class C> struct ColScale { static constexpr int value = (int)sizeof(C); };

template <class P>
struct TriArgs {
  TriDev<P> lo, up;
  const int32_t* blk_row;    // nb+1 block row starts (level-local)
  typename P::X* t;          // working vector at this level's start
  int64_t d;                 // rows of B_l
  CsrDev<P> F;               // UP mode: F_l (rows of B_l, cols of C_l)
  typename P::X* xg;         // scratch (d entries) when blocks exceed LDS
  typename P::C* fy;         // streamed UP mode: F_l y2 (d entries), formed first
  int32_t nb;
  // streamed layout (used when `blob` is set)
  const uint8_t* blob;
  const ChunkDesc* chunk;
  const int32_t* blk_chunk;  // nb+1 chunk ranges
  int32_t chunk_cap;         // max chunk bytes (multiple of 1 KiB)
  int32_t x_bytes;           // LDS bytes reserved for the block's vector (16-aligned)
  int32_t half_u;            // U chunks in half-row form: lanes l and l+32 share row l
  int32_t half_l;            // L chunks likewise
  // level 0 of an apply (streamed kernel only): DOWN reads its right-hand
  // side from the caller's vector, xin[perm[row]], instead of t; UP writes
  // its result to yout[perm[row]] instead of t.  null: use t.  perm null:
  // identity (vectors already in the permuted order).
  const typename P::O* xin;
  typename P::O* yout;
  const int32_t* perm;
  // UP with yout (single vector, streamed kernel): the sweep also writes the
  // ccopy rows of C_l, yout[perm[d + i]] = t[d + i] for i < ccopy (the
  // apply's final scatter); workgroup b takes rows b * ccopy / nb up to
  // (b + 1) * ccopy / nb, copied by its producer wave while the last chunk
  // is swept.  0: none.
  int64_t ccopy = 0;
  // DOWN (streamed kernel): the sweep also files z1 under the entries of
  // E_l, ez[p] = z1[col] for every entry p of E_l (its index in E_l's CSR
  // order), so the interface step reads them in that order instead of
  // gathering z1.  Sweep unit b owns records eunit[b] .. eunit[b + 1] - 1
  // (an even count: 16-byte aligned), record q = (erec[2q] = p,
  // erec[2q + 1] = unit-local row), p < 0 for padding; at most chunk_cap
  // bytes per unit.  Vector j writes ez + j * ldez.  null: none.
  const int32_t* erec = nullptr;
  const int32_t* eunit = nullptr;
  typename P::X* ez = nullptr;
  int64_t ldez = 0;
  // streamed UP mode: F_l y2 formed by the sweep itself, from the rows of
  // F_l that hold entries (null: read from fy, formed by a launch before).
  // Record q is unit-local row frow[q] with entries j < fw at
  // fcol/fval[j * nrec + q] (level-local C columns; padding column 0,
  // value 0); sweep unit b owns records funit[b] .. funit[b + 1] - 1.
  const int32_t* frow = nullptr;
  const int32_t* fcol = nullptr;
  const typename P::V* fval = nullptr;
  const int32_t* funit = nullptr;
  int32_t fw = 0;
  int64_t nrec = 0;
  // several vectors per launch: t and fy of vector j start at t + j * ldt
  // and fy + j * ldfy.  The streamed kernel sweeps vectors
  // ncons * blockIdx.y + c, c < ncons, in one workgroup: consumer wave c
  // holds its own block vector in LDS and all of them sweep the same staged
  // chunks (factor entries read once for ncons vectors); the other kernels
  // take vector j = blockIdx.y.
  int32_t nvec = 1;
  int32_t ncons = 1;
  int64_t ldt = 0, ldfy = 0;
};

// most consumer waves (vectors) per workgroup of the streamed sweep
constexpr int kMaxCons = 8;
// ... for elements of csize bytes and rows of ms slots: as many as the
// sweep's registers allow (a workgroup of c + 1 waves has 512 / ceil((c + 1)
// / 4) registers per lane: 168 at 8 consumers, 256 at 4, 512 at 3; the
// 16-slot float64 and the 8-or-more-slot complex128 sweeps need more than
// 168, the 12- and 16-slot complex128 ones more than 256)
__host__ __device__ constexpr int stream_max_cons(int csize, int ms) {
  return csize >= 16 ? (ms <= 4 ? kMaxCons : ms <= 10 ? 4 : 3) : (ms <= 12 ? kMaxCons : 4);
}
// LDS bytes of a streamed-sweep workgroup with c consumers: c block vectors,
// two chunk buffers and 1 KiB of slack after the second (lanes past the end
// of a stage read, and then discard, up to 63 elements beyond a section)
inline size_t stream_lds_bytes(int x_bytes, int chunk_cap, int c) {
  return (size_t)c * (size_t)x_bytes + 2 * (size_t)chunk_cap + 1024;
}

template <class P>
struct IfArgs {
  CsrDev<P> E;               // s x d
  typename P::X* t;          // working vector at this level's start
  int64_t d, s;
  int32_t k;
  const typename P::V* W;    // s x k column-major
  const typename P::C* H;    // k x k column-major, compute type
  typename P::C* partial;    // gridDim x k partial sums of W^H z2
  typename P::C* tprime;     // k: H (W^H z2), written by a second launch
  // small-level kernel only: when the next (last) level is diagonal, its
  // solve in the same pass: C-part = w * last_dinv (1/u_ii in row order)
  const typename P::D* last_dinv = nullptr;
  // level 0 of an apply: b2 read from the caller's vector, xin[perm[d + i]]
  // (perm null: identity), instead of t
  const typename P::O* xin = nullptr;
  const int32_t* perm = nullptr;
  // small-level kernel: copy W_l and H_l to LDS when they fit in max_lds
  // bytes of the workgroup's LDS (0: read them from global memory)
  int32_t stage_w = 1;
  int32_t max_lds = 65536;
  // several vectors per launch (blockIdx.y = vector j): t, partial and
  // tprime of vector j start at t + j * ldt, partial + j * ldpart and
  // tprime + j * k
  int32_t nvec = 1;
  int64_t ldt = 0, ldpart = 0;
  // z1 filed in E_l's entry order by the level's down sweep (see
  // TriArgs::erec): the E product reads ez[p] instead of t[col(p)]; vector
  // j at ez + j * ldez.  null: gather from t.
  const typename P::X* ez = nullptr;
  int64_t ldez = 0;
};

// ------------------------------------------------------------ launchers
template <class P> void launch_trisolve(const TriArgs<P>& a, int mode, int maxslot,
                                        int max_block_rows, hipStream_t st);
// streamed variant: one producer wave stages chunks into LDS, a.ncons
// consumer waves sweep them; needs a.blob, x in LDS, and maxslot <= 16
template <class P> void launch_trisolve_streamed(const TriArgs<P>& a, int mode, int maxslot,
                                                 int max_block_rows, hipStream_t st);
// maximum chunk size the streamed kernel stages (bytes): 48 copy
// iterations per lane, within the 63 loads a wave can have outstanding
// (measured: 24 -> 48 KiB took the 64^3 apply from 287 to 269 us and the
// complex128 128^3 apply from 892 to 835 us, where one workgroup per CU
// sweeps level 0; at two per CU LDS keeps level 0 at 23 KiB)
constexpr int kChunkCapMax = 49152;
template <class P> void launch_interface(const IfArgs<P>& a, hipStream_t st);
// dst[i] = src[i] rounded to V (float or bf16) as the host storage
// conversion rounds it
template <class V> void launch_store_from_double(const double* src, V* dst, int64_t n,
                                                 hipStream_t st);
// the interface step and the low-rank update of a small level (s <= 4096,
// k <= 64) in one launch; returns false (launching nothing) otherwise
template <class P> bool launch_interface_small(const IfArgs<P>& a, hipStream_t st);
// upper bound of the workgroups launch_interface uses for s interface rows
// (`partial` holds this many times k entries)
template <class P> int interface_blocks(int64_t s);
template <class P> void launch_lowrank_update(typename P::X* tc, int64_t s, int k,
                                              const typename P::V* W,
                                              const typename P::C* tprime, hipStream_t st,
                                              int nvec = 1, int64_t ldt = 0);
template <class P> void launch_gather(const typename P::O* x, const int32_t* perm,
                                      typename P::X* t, int64_t n, hipStream_t st);
template <class P> void launch_scatter(const typename P::X* t, const int32_t* perm,
                                       typename P::O* y, int64_t n, hipStream_t st);

// float64 / complex128 vector kernels for FGMRES and Arnoldi
template <class T> void launch_spmv(const int32_t* rp, const int32_t* ci, const T* v,
                                    const T* x, T* y, int64_t n, hipStream_t st);
// y = b - A x
template <class T> void launch_residual(const int32_t* rp, const int32_t* ci, const T* v,
                                        const T* x, const T* b, T* y, int64_t n, hipStream_t st);
// h[c] = sum_i conj(V[i + c ld]) w[i], c < ncol (partials then a fixed-order sum)
template <class T> void launch_multidot(const T* V, int64_t ld, int ncol, const T* w,
                                        int64_t n, T* partial, T* h, hipStream_t st);
// w -= V h (ncol columns); if hacc != null also hacc += h
template <class T> void launch_gemv_sub(const T* V, int64_t ld, int ncol, const T* h,
                                        T* w, int64_t n, T* hacc, hipStream_t st);
// out[0] = ||w||_2 (partials then fixed-order sum)
template <class T> void launch_norm(const T* w, int64_t n, double* partial, double* out,
                                   hipStream_t st);
// y = x / (*nrm)  (or zero when *nrm == 0)
// one Arnoldi step's bookkeeping on the device (see kernels.hip)
template <class T> void launch_arnoldi_step(const T* h, int cnt, const double* nrm, T* Scol,
                                            double* nd, double* flag, const T* w, T* y, int64_t n,
                                            hipStream_t st);
template <class T> void launch_scale_inv(const T* x, const double* nrm, T* y, int64_t n,
                                         hipStream_t st);
// x += Z y (ncol columns)
template <class T> void launch_gemv_add(const T* Z, int64_t ld, int ncol, const T* y,
                                        T* x, int64_t n, hipStream_t st);
// Y = V G with V n x m (ld), G m x k column-major (host-computed), Y n x k (ldy)
template <class T> void launch_gemm_small(const T* V, int64_t ld, int m, const T* G, int k,
                                          T* Y, int64_t ldy, int64_t n, hipStream_t st);
template <class T> void launch_fill(T* x, T v, int64_t n, hipStream_t st);
// V[:, c] (column-major, ld) = Y[:, c], c < k, for a row-major float32
// block Y with row stride ldy >= k
template <class T> void launch_rows_to_cols(const float* Y, int64_t s, int k, int ldy, T* V,
                                            int64_t ld, hipStream_t st);
// out = a - b (n entries)
template <class T> void launch_sub(const T* a, const T* b, T* out, int64_t n, hipStream_t st);
// y[i] = x[perm[i]] (gather into reordered numbering) / y[perm[i]] = x[i]
template <class T> void launch_permute(const T* x, const int32_t* perm, T* y, int64_t n,
                                       bool scatter, hipStream_t st);
template <class T> void launch_copy(const T* x, T* y, int64_t n, hipStream_t st);
// inner GMRES at the root level: c (m) minimising ||beta e1 - Hbar c|| for
// the Arnoldi columns h ((m+1) x m, column-major), subdiagonal norms sub and
// pre-orthogonalisation norms wn (m+1 each, entry 0 unused)
constexpr int kInnerMax = 16;
template <class T> void launch_inner_lsq(const T* h, const double* sub, const double* wn,
                                         const double* beta, int m, T* c, hipStream_t st);

}  // namespace gs
