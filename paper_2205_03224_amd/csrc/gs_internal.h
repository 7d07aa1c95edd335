// Internal declarations of libgemslr (host side).  Nothing here is part of
// the C ABI; see include/gemslr.h for that.
#pragma once

#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "gemslr.h"

namespace gs {

using cplx = std::complex<double>;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

inline double absval(double x) { return x < 0 ? -x : x; }
inline double absval(const cplx& x) { return std::abs(x); }
inline double realpart(double x) { return x; }
inline double realpart(const cplx& x) { return x.real(); }
inline double conjv(double x) { return x; }
inline cplx conjv(const cplx& x) { return std::conj(x); }
template <class T> inline bool finite(const T& x) {
  return std::isfinite(realpart(x)) && std::isfinite(std::imag(std::complex<double>(x)));
}

// Compressed sparse rows; columns sorted ascending in every row.
template <class T>
struct CSR {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rp{0};
  std::vector<int32_t> ci;
  std::vector<T> v;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// --------------------------------------------------------------- partition
struct Partition {
  std::vector<int64_t> perm;          // perm[new] = old
  int L = 0;                          // levels with a Schur complement
  std::vector<int64_t> level_start;   // L+2 entries
  std::vector<std::vector<int64_t>> blocks;  // L+1 lists of global boundaries
};

// Validate a CSR (sorted, in range, diagonal present); throws Error.
void validate_csr(int64_t n, const int64_t* rp, const int32_t* ci,
                  bool need_diag);

Partition partition_grid(int ndim, const int32_t* dims, int nparts,
                         int levels, int64_t n, const int64_t* rp,
                         const int32_t* ci);
// Nested dissection by breadth-first level structures (no coordinates
// needed); nparts a power of two.
Partition partition_graph(int nparts, int levels, int64_t n, const int64_t* rp,
                          const int32_t* ci);
// A partition given by the caller (perm[new] = old, L + 2 segment starts),
// checked against A's pattern: every segment non-empty, and B_l (l < L)
// block diagonal.  Blocks given as global boundaries per segment (block_ptr,
// block_count as gs_partition_grid writes them) or, when block_ptr is null,
// the connected components of each segment's rows in the symmetrised graph
// of A, which must each be contiguous in perm.  Throws Error(GS_EINVAL).
Partition user_partition(int64_t n, const int64_t* rp, const int32_t* ci, const int64_t* perm,
                         const int64_t* level_start, int L, const int64_t* block_ptr,
                         const int64_t* block_count);

// --------------------------------------------------------------- ILU
template <class T>
void ilu0(const CSR<T>& B, CSR<T>& L, CSR<T>& U);
template <class T>
void ilut(const CSR<T>& B, double tau, int lfil, CSR<T>& L, CSR<T>& U);

// --------------------------------------------------------------- levels
// One level in permuted numbering; level L (the last separator) has s = 0.
template <class T>
struct HostLevel {
  int64_t start = 0, d = 0, s = 0;
  std::vector<int64_t> blocks;  // nb+1 boundaries relative to start
  CSR<T> L, U, E, F;            // level-local numbering
  int k = 0;
  std::vector<T> W, H;          // s x k and k x k, column-major
  // W held only by the device engine (in this precision, exactly) and
  // fetched into W when the host needs it; W is empty meanwhile
  bool w_on_device = false;
  int arnoldi_cycles = 0, arnoldi_matvecs = 0, arnoldi_converged = 0;
};

template <class T>
struct HostSetup {
  int64_t n = 0;
  std::vector<int64_t> perm;
  std::vector<HostLevel<T>> lv;  // L+1 entries
  CSR<T> A;                      // original matrix
  CSR<T> Ap;                     // P^T A P
  int L() const { return (int)lv.size() - 1; }
};

// P^T A P for perm[new] = old, rows sorted by column.
template <class T>
CSR<T> permute(const CSR<T>& A, const std::vector<int64_t>& perm);

// Permute A and cut it into the level structure of `part`; the last level
// keeps only its diagonal blocks (block Jacobi).
template <class T>
void extract_levels(const CSR<T>& A, const Partition& part, HostSetup<T>& S);

// Factor every diagonal block of every level with `nthreads` host threads.
template <class T>
// shift: added to every diagonal entry of each block before its ILU (the
// complex shift of the Helmholtz experiments; zero otherwise)
void factor_levels(HostSetup<T>& S, int kind, double tau, int lfil,
                   int nthreads, T shift = T(0));

// --------------------------------------------------------------- small dense
// Complex Schur decomposition A = Q T Q^H of an m x m column-major matrix by
// Householder reduction to Hessenberg form and shifted QR iteration.
// On return a holds T (upper triangular) and q holds Q.
void schur_complex(int m, std::vector<cplx>& a, std::vector<cplx>& q);
// The same for a real m x m column-major matrix a: the real Schur form by
// the double-shift QR iteration, its 2x2 blocks (complex-conjugate pairs)
// then made triangular, so that t (upper triangular) and q (unitary) are a
// complex Schur form a = q t q^H.
void schur_real(int m, const std::vector<double>& a, std::vector<cplx>& t, std::vector<cplx>& q);
// Reorder a complex Schur form so that the positions flagged in `sel` come
// first (adjacent swaps by plane rotations); sel is permuted along.
void schur_reorder(int m, std::vector<cplx>& t, std::vector<cplx>& q,
                   std::vector<int>& sel);
// Eigenvectors of an upper triangular k x k matrix (columns, unit 2-norm).
void triu_eigvecs(int k, const std::vector<cplx>& t, std::vector<cplx>& y);
// Mask of the wanted Ritz values (ordered by |theta/(1-theta)|, ties to
// larger |theta|, then lower index); with real_pairs, conjugate partners are
// added so that no pair is split.
std::vector<int> select_wanted(const std::vector<cplx>& theta, int k,
                               bool real_pairs);
// H = (I - R)^{-1} - I for a k x k column-major R (LU with partial pivoting);
// throws Error(GS_ESINGULAR) when an eigenvalue of R is within 1e-12 of 1.
template <class T>
std::vector<T> correction_matrix(int k, const std::vector<T>& R,
                                 const std::vector<cplx>& theta);

// SplitMix64 start vector: v[i] = 2 u_i - 1, u_i the top 53 bits of the i-th
// output of SplitMix64 seeded with `seed`.
void start_vector(uint64_t seed, int64_t n, double* v);

}  // namespace gs
