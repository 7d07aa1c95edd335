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
  // Real and imaginary parts in separate column-major arrays, so that the
  // column and Schur-vector updates below are contiguous loops the compiler
  // vectorises; the arithmetic is the same as with std::complex.
  const size_t mm = (size_t)m * m;
  std::vector<double> Ar(mm), Ai(mm), Qr(mm, 0.0), Qi(mm, 0.0);
  for (size_t e = 0; e < mm; ++e) {
    Ar[e] = a[e].real();
    Ai[e] = a[e].imag();
  }
  for (int i = 0; i < m; ++i) Qr[(size_t)i * m + i] = 1.0;
  auto ix = [m](int i, int j) { return (size_t)j * m + i; };
  if (m > 1) {
    // --- Householder reduction to Hessenberg form: A <- P A P, Q <- Q P,
    // P = I - 2 v v^H / |v|^2
    std::vector<double> vr(m), vi(m), wr(m), wi(m);
    for (int k = 0; k + 2 < m; ++k) {
      double xn = 0;
      for (int i = k + 1; i < m; ++i) xn += Ar[ix(i, k)] * Ar[ix(i, k)] + Ai[ix(i, k)] * Ai[ix(i, k)];
      xn = std::sqrt(xn);
      if (xn == 0) continue;
      const double x0r = Ar[ix(k + 1, k)], x0i = Ai[ix(k + 1, k)];
      const double x0a = std::hypot(x0r, x0i);
      const double phr = x0a > 0 ? x0r / x0a : 1.0, phi = x0a > 0 ? x0i / x0a : 0.0;
      for (int i = k + 1; i < m; ++i) {
        vr[i] = Ar[ix(i, k)];
        vi[i] = Ai[ix(i, k)];
      }
      vr[k + 1] += phr * xn;
      vi[k + 1] += phi * xn;
      double vn = 0;
      for (int i = k + 1; i < m; ++i) vn += vr[i] * vr[i] + vi[i] * vi[i];
      if (vn == 0) continue;
      const double f = 2.0 / vn;
      // A <- P A: column j -= v (v^H A_j) f
      for (int j = 0; j < m; ++j) {
        const double* cr = &Ar[ix(0, j)];
        const double* ci = &Ai[ix(0, j)];
        double sr = 0, si = 0;
        for (int i = k + 1; i < m; ++i) {  // conj(v) * a
          sr += vr[i] * cr[i] + vi[i] * ci[i];
          si += vr[i] * ci[i] - vi[i] * cr[i];
        }
        sr *= f;
        si *= f;
        double* dr = &Ar[ix(0, j)];
        double* di = &Ai[ix(0, j)];
        for (int i = k + 1; i < m; ++i) {
          dr[i] -= vr[i] * sr - vi[i] * si;
          di[i] -= vr[i] * si + vi[i] * sr;
        }
      }
      // M <- M P for M = A, Q: w = M v, then column j -= w conj(v_j) f
      for (int which = 0; which < 2; ++which) {
        std::vector<double>& Mr = which ? Qr : Ar;
        std::vector<double>& Mi = which ? Qi : Ai;
        std::fill(wr.begin(), wr.end(), 0.0);
        std::fill(wi.begin(), wi.end(), 0.0);
        for (int j = k + 1; j < m; ++j) {
          const double* cr = &Mr[ix(0, j)];
          const double* ci = &Mi[ix(0, j)];
          const double br = vr[j], bi = vi[j];
          for (int i = 0; i < m; ++i) {
            wr[i] += cr[i] * br - ci[i] * bi;
            wi[i] += cr[i] * bi + ci[i] * br;
          }
        }
        for (int j = k + 1; j < m; ++j) {
          const double br = vr[j] * f, bi = -vi[j] * f;  // conj(v_j) f
          double* dr = &Mr[ix(0, j)];
          double* di = &Mi[ix(0, j)];
          for (int i = 0; i < m; ++i) {
            dr[i] -= wr[i] * br - wi[i] * bi;
            di[i] -= wr[i] * bi + wi[i] * br;
          }
        }
      }
      for (int i = k + 2; i < m; ++i) Ar[ix(i, k)] = Ai[ix(i, k)] = 0.0;
    }
    // --- shifted QR on the Hessenberg matrix
    auto absA = [&](int i, int j) { return std::hypot(Ar[ix(i, j)], Ai[ix(i, j)]); };
    int hi = m - 1;
    int iter = 0, total = 0;
    while (hi > 0) {
      // find the start of the active unreduced block
      int lo = hi;
      while (lo > 0) {
        const double sub = absA(lo, lo - 1);
        double dd = absA(lo - 1, lo - 1) + absA(lo, lo);
        if (dd == 0) dd = 1.0;
        if (sub <= kEps * dd) {
          Ar[ix(lo, lo - 1)] = Ai[ix(lo, lo - 1)] = 0.0;
          break;
        }
        --lo;
      }
      if (lo == hi) {
        --hi;
        iter = 0;
        continue;
      }
      if (++total > 100 * m) throw Error(GS_EINVAL, "Schur QR iteration did not converge");
      ++iter;
      // Wilkinson shift from the trailing 2x2 of the active block
      cplx sigma;
      if (iter % 11 == 10) {
        sigma = cplx(Ar[ix(hi, hi)], Ai[ix(hi, hi)]) + 0.75 * absA(hi, hi - 1);
      } else {
        const cplx aa(Ar[ix(hi - 1, hi - 1)], Ai[ix(hi - 1, hi - 1)]);
        const cplx bb(Ar[ix(hi - 1, hi)], Ai[ix(hi - 1, hi)]);
        const cplx cc(Ar[ix(hi, hi - 1)], Ai[ix(hi, hi - 1)]);
        const cplx dd(Ar[ix(hi, hi)], Ai[ix(hi, hi)]);
        const cplx tr2 = (aa + dd) * 0.5;
        const cplx disc = std::sqrt((aa - dd) * (aa - dd) * 0.25 + bb * cc);
        const cplx e1 = tr2 + disc, e2 = tr2 - disc;
        sigma = (std::abs(e1 - dd) < std::abs(e2 - dd)) ? e1 : e2;
      }
      // implicit single-shift bulge chase on rows/cols lo..hi
      double xr = Ar[ix(lo, lo)] - sigma.real(), xi = Ai[ix(lo, lo)] - sigma.imag();
      double yr = Ar[ix(lo + 1, lo)], yi = Ai[ix(lo + 1, lo)];
      for (int k = lo; k < hi; ++k) {
        const double r = std::sqrt(xr * xr + xi * xi + yr * yr + yi * yi);
        double cr = 1, ci = 0, sr = 0, si = 0;
        if (r != 0) {
          cr = xr / r;
          ci = xi / r;
          sr = yr / r;
          si = yi / r;
        }
        // rows k, k+1 <- G^H rows, G^H = [[conj c, conj s], [-s, c]]
        for (int j = std::max(lo, k - 1); j < m; ++j) {
          const size_t p0 = ix(k, j), p1 = p0 + 1;
          const double pr = Ar[p0], pi = Ai[p0], tr = Ar[p1], ti = Ai[p1];
          Ar[p0] = (cr * pr + ci * pi) + (sr * tr + si * ti);
          Ai[p0] = (cr * pi - ci * pr) + (sr * ti - si * tr);
          Ar[p1] = -(sr * pr - si * pi) + (cr * tr - ci * ti);
          Ai[p1] = -(sr * pi + si * pr) + (cr * ti + ci * tr);
        }
        if (k > lo) Ar[ix(k + 1, k - 1)] = Ai[ix(k + 1, k - 1)] = 0.0;  // the bulge just annihilated
        // cols k, k+1 <- cols G, G = [[c, -conj s], [s, conj c]]
        const int imax = std::min(k + 2, hi);
        for (int which = 0; which < 2; ++which) {
          double* Pr = which ? &Qr[ix(0, k)] : &Ar[ix(0, k)];
          double* Pi = which ? &Qi[ix(0, k)] : &Ai[ix(0, k)];
          double* Tr = Pr + m;
          double* Ti = Pi + m;
          const int n = which ? m : imax + 1;
          for (int i = 0; i < n; ++i) {
            const double pr = Pr[i], pi = Pi[i], tr = Tr[i], ti = Ti[i];
            Pr[i] = (pr * cr - pi * ci) + (tr * sr - ti * si);
            Pi[i] = (pr * ci + pi * cr) + (tr * si + ti * sr);
            Tr[i] = -(pr * sr + pi * si) + (tr * cr + ti * ci);
            Ti[i] = -(pi * sr - pr * si) + (ti * cr - tr * ci);
          }
        }
        if (k + 1 < hi) {
          xr = Ar[ix(k + 1, k)];
          xi = Ai[ix(k + 1, k)];
          yr = Ar[ix(k + 2, k)];
          yi = Ai[ix(k + 2, k)];
        }
      }
    }
  }
  q.assign(mm, cplx(0));
  for (size_t e = 0; e < mm; ++e) {
    a[e] = cplx(Ar[e], Ai[e]);
    q[e] = cplx(Qr[e], Qi[e]);
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
