// Small dense linear algebra on the host for the low-rank setup: the
// Rayleigh-quotient matrices of thick-restart Arnoldi are at most a few
// hundred wide, so they are decomposed here rather than on the GPU.
//
// Complex Schur form: Householder reduction to upper Hessenberg form, then
// the single-shift QR algorithm with Wilkinson shifts and deflation, chasing
// the bulge with plane rotations (Golub & Van Loan, Matrix Computations,
// Sec. 7.4-7.5, complex version).  Reordering swaps adjacent diagonal entries
// with one plane rotation each (Bai & Demmel's swap in the 1x1 case).
#include <algorithm>
#include <cmath>
#include <limits>

#include "gs_internal.h"

namespace gs {

namespace {
inline cplx& at(std::vector<cplx>& a, int m, int i, int j) { return a[(size_t)j * m + i]; }
inline cplx at(const std::vector<cplx>& a, int m, int i, int j) { return a[(size_t)j * m + i]; }
const double kEps = std::numeric_limits<double>::epsilon();
}  // namespace

void schur_complex(int m, std::vector<cplx>& a, std::vector<cplx>& q) {
  q.assign((size_t)m * m, cplx(0));
  for (int i = 0; i < m; ++i) at(q, m, i, i) = 1.0;
  if (m <= 1) return;
  // --- Householder reduction to Hessenberg form: A <- P A P, Q <- Q P
  std::vector<cplx> v(m);
  for (int k = 0; k + 2 < m; ++k) {
    double xn = 0;
    for (int i = k + 1; i < m; ++i) xn += std::norm(at(a, m, i, k));
    xn = std::sqrt(xn);
    if (xn == 0) continue;
    cplx x0 = at(a, m, k + 1, k);
    cplx ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cplx(1);
    for (int i = 0; i < m; ++i) v[i] = 0;
    for (int i = k + 1; i < m; ++i) v[i] = at(a, m, i, k);
    v[k + 1] += ph * xn;
    double vn = 0;
    for (int i = k + 1; i < m; ++i) vn += std::norm(v[i]);
    if (vn == 0) continue;
    // A <- (I - 2 v v^H / vn) A
    for (int j = 0; j < m; ++j) {
      cplx s = 0;
      for (int i = k + 1; i < m; ++i) s += std::conj(v[i]) * at(a, m, i, j);
      s *= 2.0 / vn;
      for (int i = k + 1; i < m; ++i) at(a, m, i, j) -= v[i] * s;
    }
    // A <- A (I - 2 v v^H / vn), Q likewise
    for (std::vector<cplx>* M : {&a, &q}) {
      for (int i = 0; i < m; ++i) {
        cplx s = 0;
        for (int j = k + 1; j < m; ++j) s += at(*M, m, i, j) * v[j];
        s *= 2.0 / vn;
        for (int j = k + 1; j < m; ++j) at(*M, m, i, j) -= s * std::conj(v[j]);
      }
    }
    for (int i = k + 2; i < m; ++i) at(a, m, i, k) = 0;
  }
  // --- shifted QR on the Hessenberg matrix
  int hi = m - 1;
  int iter = 0, total = 0;
  while (hi > 0) {
    // find the start of the active unreduced block
    int lo = hi;
    while (lo > 0) {
      double sub = std::abs(at(a, m, lo, lo - 1));
      double dd = std::abs(at(a, m, lo - 1, lo - 1)) + std::abs(at(a, m, lo, lo));
      if (dd == 0) dd = 1.0;
      if (sub <= kEps * dd) { at(a, m, lo, lo - 1) = 0; break; }
      --lo;
    }
    if (lo == hi) { --hi; iter = 0; continue; }
    if (++total > 100 * m) throw Error(GS_EINVAL, "Schur QR iteration did not converge");
    ++iter;
    // Wilkinson shift from the trailing 2x2 of the active block
    cplx sigma;
    if (iter % 11 == 10) {
      sigma = at(a, m, hi, hi) + 0.75 * std::abs(at(a, m, hi, hi - 1));
    } else {
      cplx aa = at(a, m, hi - 1, hi - 1), bb = at(a, m, hi - 1, hi);
      cplx cc = at(a, m, hi, hi - 1), dd = at(a, m, hi, hi);
      cplx tr2 = (aa + dd) * 0.5;
      cplx disc = std::sqrt((aa - dd) * (aa - dd) * 0.25 + bb * cc);
      cplx e1 = tr2 + disc, e2 = tr2 - disc;
      sigma = (std::abs(e1 - dd) < std::abs(e2 - dd)) ? e1 : e2;
    }
    // implicit single-shift bulge chase on rows/cols lo..hi
    cplx x = at(a, m, lo, lo) - sigma;
    cplx y = at(a, m, lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      double r = std::sqrt(std::norm(x) + std::norm(y));
      cplx c, s;
      if (r == 0) { c = 1; s = 0; }
      else { c = x / r; s = y / r; }
      // rows k, k+1 <- G^H rows, G^H = [[conj c, conj s], [-s, c]]
      for (int j = std::max(lo, k - 1); j < m; ++j) {
        cplx p = at(a, m, k, j), t = at(a, m, k + 1, j);
        at(a, m, k, j) = std::conj(c) * p + std::conj(s) * t;
        at(a, m, k + 1, j) = -s * p + c * t;
      }
      if (k > lo) at(a, m, k + 1, k - 1) = 0;  // the bulge just annihilated
      // cols k, k+1 <- cols G, G = [[c, -conj s], [s, conj c]]
      int imax = std::min(k + 2, hi);
      for (int i = 0; i <= imax; ++i) {
        cplx p = at(a, m, i, k), t = at(a, m, i, k + 1);
        at(a, m, i, k) = p * c + t * s;
        at(a, m, i, k + 1) = -p * std::conj(s) + t * std::conj(c);
      }
      for (int i = 0; i < m; ++i) {
        cplx p = at(q, m, i, k), t = at(q, m, i, k + 1);
        at(q, m, i, k) = p * c + t * s;
        at(q, m, i, k + 1) = -p * std::conj(s) + t * std::conj(c);
      }
      if (k + 1 < hi) {
        x = at(a, m, k + 1, k);
        y = at(a, m, k + 2, k);
      }
    }
  }
  for (int j = 0; j < m; ++j)
    for (int i = j + 1; i < m; ++i) at(a, m, i, j) = 0;
}

void schur_reorder(int m, std::vector<cplx>& t, std::vector<cplx>& q,
                   std::vector<int>& sel) {
  int ks = 0;
  for (int j = 0; j < m; ++j) {
    if (!sel[j]) continue;
    for (int p = j - 1; p >= ks; --p) {
      // swap diagonal entries p and p+1
      cplx t11 = at(t, m, p, p), t22 = at(t, m, p + 1, p + 1), t12 = at(t, m, p, p + 1);
      cplx vx = t12, vy = t22 - t11;
      double r = std::sqrt(std::norm(vx) + std::norm(vy));
      if (r > 0) {
        cplx c = vx / r, s = vy / r;
        // rows p, p+1 <- Z^H rows, Z = [[c, -conj s], [s, conj c]]
        for (int jj = p; jj < m; ++jj) {
          cplx a1 = at(t, m, p, jj), a2 = at(t, m, p + 1, jj);
          at(t, m, p, jj) = std::conj(c) * a1 + std::conj(s) * a2;
          at(t, m, p + 1, jj) = -s * a1 + c * a2;
        }
        for (int i = 0; i <= p + 1; ++i) {
          cplx a1 = at(t, m, i, p), a2 = at(t, m, i, p + 1);
          at(t, m, i, p) = a1 * c + a2 * s;
          at(t, m, i, p + 1) = -a1 * std::conj(s) + a2 * std::conj(c);
        }
        for (int i = 0; i < m; ++i) {
          cplx a1 = at(q, m, i, p), a2 = at(q, m, i, p + 1);
          at(q, m, i, p) = a1 * c + a2 * s;
          at(q, m, i, p + 1) = -a1 * std::conj(s) + a2 * std::conj(c);
        }
      }
      at(t, m, p, p) = t22;
      at(t, m, p + 1, p + 1) = t11;
      at(t, m, p + 1, p) = 0;
      std::swap(sel[p], sel[p + 1]);
    }
    ++ks;
  }
}

void triu_eigvecs(int k, const std::vector<cplx>& t, std::vector<cplx>& y) {
  y.assign((size_t)k * k, cplx(0));
  double tn = 0;
  for (auto& x : t) tn = std::max(tn, std::abs(x));
  const double small = std::max(tn, 1e-300) * kEps;
  for (int i = 0; i < k; ++i) {
    at(y, k, i, i) = 1.0;
    const cplx lam = at(t, k, i, i);
    for (int r = i - 1; r >= 0; --r) {
      cplx s = 0;
      for (int c = r + 1; c <= i; ++c) s += at(t, k, r, c) * at(y, k, c, i);
      cplx den = at(t, k, r, r) - lam;
      if (std::abs(den) < small) den = small;
      at(y, k, r, i) = -s / den;
    }
    double nr = 0;
    for (int r = 0; r <= i; ++r) nr += std::norm(at(y, k, r, i));
    nr = std::sqrt(nr);
    for (int r = 0; r <= i; ++r) at(y, k, r, i) /= nr;
  }
}

std::vector<int> select_wanted(const std::vector<cplx>& theta, int k,
                               bool real_pairs) {
  const int m = (int)theta.size();
  std::vector<int> sel(m, 0);
  k = std::min(k, m);
  if (k <= 0) return sel;
  std::vector<double> w(m);
  for (int i = 0; i < m; ++i) {
    cplx den = 1.0 - theta[i];
    w[i] = std::abs(den) == 0 ? std::numeric_limits<double>::infinity()
                              : std::abs(theta[i] / den);
  }
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    if (w[a] != w[b]) return w[a] > w[b];
    double ta = std::abs(theta[a]), tb = std::abs(theta[b]);
    if (ta != tb) return ta > tb;
    return a < b;
  });
  for (int i = 0; i < k; ++i) sel[order[i]] = 1;
  if (real_pairs) {
    // eigenvalues of a real matrix computed in complex arithmetic: a value is
    // taken as non-real when its imaginary part is above rounding level
    double scale = 0;
    for (auto& x : theta) scale = std::max(scale, std::abs(x));
    const double tol = 1e-10 * std::max(scale, 1e-300);
    std::vector<int> add;
    for (int i = 0; i < m; ++i) {
      if (!sel[i] || std::abs(theta[i].imag()) <= tol) continue;
      int best = -1;
      double bd = 0;
      for (int j = 0; j < m; ++j) {
        if (j == i) continue;
        double dd = std::abs(theta[j] - std::conj(theta[i]));
        if (best < 0 || dd < bd) { best = j; bd = dd; }
      }
      if (best >= 0) add.push_back(best);
    }
    for (int j : add) sel[j] = 1;
  }
  return sel;
}

template <class T>
std::vector<T> correction_matrix(int k, const std::vector<T>& R,
                                 const std::vector<cplx>& theta) {
  for (auto& th : theta)
    if (std::abs(1.0 - th) < 1e-12)
      throw Error(GS_ESINGULAR, "Ritz value within 1e-12 of 1: I - R_k is singular");
  // solve (I - R) X = I by Gaussian elimination with partial pivoting
  std::vector<T> M((size_t)k * k), X((size_t)k * k, T(0));
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i)
      M[(size_t)j * k + i] = (i == j ? T(1) : T(0)) - R[(size_t)j * k + i];
  for (int i = 0; i < k; ++i) X[(size_t)i * k + i] = T(1);
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int i = c + 1; i < k; ++i)
      if (absval(M[(size_t)c * k + i]) > absval(M[(size_t)c * k + piv])) piv = i;
    if (absval(M[(size_t)c * k + piv]) == 0)
      throw Error(GS_ESINGULAR, "I - R_k is singular");
    if (piv != c) {
      for (int j = 0; j < k; ++j) {
        std::swap(M[(size_t)j * k + c], M[(size_t)j * k + piv]);
        std::swap(X[(size_t)j * k + c], X[(size_t)j * k + piv]);
      }
    }
    for (int i = c + 1; i < k; ++i) {
      T f = M[(size_t)c * k + i] / M[(size_t)c * k + c];
      if (absval(f) == 0) continue;
      for (int j = c; j < k; ++j) M[(size_t)j * k + i] -= f * M[(size_t)j * k + c];
      for (int j = 0; j < k; ++j) X[(size_t)j * k + i] -= f * X[(size_t)j * k + c];
    }
  }
  for (int j = 0; j < k; ++j)
    for (int i = k - 1; i >= 0; --i) {
      T s = X[(size_t)j * k + i];
      for (int c = i + 1; c < k; ++c) s -= M[(size_t)c * k + i] * X[(size_t)j * k + c];
      X[(size_t)j * k + i] = s / M[(size_t)i * k + i];
    }
  for (int i = 0; i < k; ++i) X[(size_t)i * k + i] -= T(1);
  return X;
}

template std::vector<double> correction_matrix<double>(int, const std::vector<double>&,
                                                       const std::vector<cplx>&);
template std::vector<cplx> correction_matrix<cplx>(int, const std::vector<cplx>&,
                                                   const std::vector<cplx>&);

}  // namespace gs
