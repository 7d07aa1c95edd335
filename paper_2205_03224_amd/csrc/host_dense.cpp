// Small dense linear algebra on the host for the low-rank setup: the
// Rayleigh-quotient matrices of thick-restart Arnoldi are at most a few
// hundred wide, so they are decomposed here rather than on the GPU.
//
// Complex Schur form: Householder reduction to upper Hessenberg form, then
// the single-shift QR algorithm with Wilkinson shifts and deflation, chasing
// the bulge with plane rotations (Golub & Van Loan, Matrix Computations,
// Sec. 7.4-7.5, complex version).  Reordering swaps adjacent diagonal entries
// with one plane rotation each (Bai & Demmel's swap in the 1x1 case).
// Real matrices take the real double-shift iteration (schur_real) and are
// then brought to the same complex triangular form.
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

void schur_real(int m, const std::vector<double>& a, std::vector<cplx>& t, std::vector<cplx>& q) {
  // A real matrix: the real Schur form A = Qr Tr Qr^T (Tr quasi-upper
  // triangular, a 2x2 diagonal block per complex-conjugate pair) by the
  // Francis double-shift QR algorithm (Golub & Van Loan, Sec. 7.5.5-7.5.6),
  // in real arithmetic, then each 2x2 block made triangular by a 2x2 unitary
  // transformation, so that A = Q T Q^H with T upper triangular as from
  // schur_complex.  About a third of the arithmetic of the complex
  // single-shift iteration on the same matrix.
  const size_t mm = (size_t)m * m;
  std::vector<double> H(a.begin(), a.begin() + mm), Z(mm, 0.0);
  for (int i = 0; i < m; ++i) Z[(size_t)i * m + i] = 1.0;
  auto ix = [m](int i, int j) { return (size_t)j * m + i; };
  // apply the reflector P = I - f v v^T (v of length len at rows r0..) to
  // rows r0.. of columns c0..c1-1 of H, and to columns r0.. of rows 0..i1-1
  // of H and of all rows of Z
  auto refl_rows = [&](const double* v, int len, int r0, int c0, int c1, double f) {
    for (int j = c0; j < c1; ++j) {
      double* col = &H[ix(r0, j)];
      double sdot = 0;
      for (int u = 0; u < len; ++u) sdot += v[u] * col[u];
      sdot *= f;
      for (int u = 0; u < len; ++u) col[u] -= sdot * v[u];
    }
  };
  auto refl_cols = [&](std::vector<double>& M, const double* v, int len, int r0, int i1, double f) {
    double* cols[3];
    for (int u = 0; u < len; ++u) cols[u] = &M[ix(0, r0 + u)];
    for (int i = 0; i < i1; ++i) {
      double sdot = 0;
      for (int u = 0; u < len; ++u) sdot += cols[u][i] * v[u];
      sdot *= f;
      for (int u = 0; u < len; ++u) cols[u][i] -= sdot * v[u];
    }
  };
  if (m > 2) {
    // Householder reduction to upper Hessenberg form
    std::vector<double> v(m), w(m);
    for (int k = 0; k + 2 < m; ++k) {
      double xn = 0;
      for (int i = k + 1; i < m; ++i) xn += H[ix(i, k)] * H[ix(i, k)];
      xn = std::sqrt(xn);
      if (xn == 0) continue;
      const int len = m - k - 1;
      for (int i = 0; i < len; ++i) v[i] = H[ix(k + 1 + i, k)];
      v[0] += v[0] >= 0 ? xn : -xn;
      double vn = 0;
      for (int i = 0; i < len; ++i) vn += v[i] * v[i];
      const double f = 2.0 / vn;
      // rows k+1.. of every column (columns < k are zero there already)
      for (int j = k; j < m; ++j) {
        double* col = &H[ix(k + 1, j)];
        double sdot = 0;
        for (int i = 0; i < len; ++i) sdot += v[i] * col[i];
        sdot *= f;
        for (int i = 0; i < len; ++i) col[i] -= sdot * v[i];
      }
      // columns k+1.. of every row of H and Z: w = M v, then M -= f w v^T
      for (int which = 0; which < 2; ++which) {
        std::vector<double>& M = which ? Z : H;
        std::fill(w.begin(), w.end(), 0.0);
        for (int u = 0; u < len; ++u) {
          const double* col = &M[ix(0, k + 1 + u)];
          const double vu = v[u];
          for (int i = 0; i < m; ++i) w[i] += col[i] * vu;
        }
        for (int u = 0; u < len; ++u) {
          double* col = &M[ix(0, k + 1 + u)];
          const double vu = v[u] * f;
          for (int i = 0; i < m; ++i) col[i] -= w[i] * vu;
        }
      }
      for (int i = k + 2; i < m; ++i) H[ix(i, k)] = 0.0;
    }
  }
  // rotation [[c, s], [-s, c]] applied to rows i, i+1 (columns c0..) and its
  // transpose to columns i, i+1 (rows 0..r1-1 of H, all of Z)
  auto rot = [&](int i, double c, double sn, int c0, int r1) {
    for (int j = c0; j < m; ++j) {
      const double x = H[ix(i, j)], y = H[ix(i + 1, j)];
      H[ix(i, j)] = c * x + sn * y;
      H[ix(i + 1, j)] = -sn * x + c * y;
    }
    for (int which = 0; which < 2; ++which) {
      std::vector<double>& M = which ? Z : H;
      double* p = &M[ix(0, i)];
      double* q2 = &M[ix(0, i + 1)];
      const int n = which ? m : r1;
      for (int r = 0; r < n; ++r) {
        const double x = p[r], y = q2[r];
        p[r] = c * x + sn * y;
        q2[r] = -sn * x + c * y;
      }
    }
  };
  // a 2x2 diagonal block at (i, i) with real eigenvalues: split it with the
  // rotation that maps an eigenvector to e_1
  auto split2 = [&](int i) {
    const double p = H[ix(i, i)], b = H[ix(i, i + 1)], c = H[ix(i + 1, i)], d = H[ix(i + 1, i + 1)];
    const double half = 0.5 * (p - d);
    const double disc = half * half + b * c;
    if (c == 0.0 || disc < 0.0) return false;
    // eigenvalue farther from d first (the stable root), eigenvector
    // (lambda - d, c)
    const double root = std::sqrt(disc);
    const double lam = d + half + (half >= 0 ? root : -root);
    double x = lam - d, y = c;
    const double r = std::hypot(x, y);
    if (r == 0.0) return false;
    x /= r;
    y /= r;
    rot(i, x, y, i, std::min(i + 2, m));
    H[ix(i + 1, i)] = 0.0;
    return true;
  };
  int hi = m - 1, iter = 0, total = 0;
  while (hi > 0) {
    int lo = hi;
    while (lo > 0) {
      double dd = std::fabs(H[ix(lo - 1, lo - 1)]) + std::fabs(H[ix(lo, lo)]);
      if (dd == 0) dd = 1.0;
      if (std::fabs(H[ix(lo, lo - 1)]) <= kEps * dd) {
        H[ix(lo, lo - 1)] = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (lo == hi - 1) {
      // a 2x2 block: split when its eigenvalues are real, else keep it
      split2(hi - 1);
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++total > 100 * m) throw Error(GS_EINVAL, "real Schur QR iteration did not converge");
    ++iter;
    // shifts s1 = (r1, i1), s2 = (r2, i2): the eigenvalues of the trailing
    // 2x2 (a real pair replaced by the one nearer H(hi, hi), taken twice),
    // exceptional ones every 11th iteration without deflation
    double r1, i1, r2, i2;
    {
      double p, b, c, d;
      if (iter % 11 == 10) {
        const double e = std::fabs(H[ix(hi, hi - 1)]) + std::fabs(H[ix(hi - 1, hi - 2)]);
        p = 0.75 * e + H[ix(hi, hi)];
        b = -0.4375 * e;
        c = e;
        d = p;
      } else {
        p = H[ix(hi - 1, hi - 1)];
        b = H[ix(hi - 1, hi)];
        c = H[ix(hi, hi - 1)];
        d = H[ix(hi, hi)];
      }
      const double half = 0.5 * (p - d);
      const double disc = half * half + b * c;
      if (disc >= 0.0) {
        const double root = std::sqrt(disc);
        const double e1 = d + half + root, e2 = d + half - root;
        const double near = std::fabs(e1 - d) <= std::fabs(e2 - d) ? e1 : e2;
        r1 = r2 = near;
        i1 = i2 = 0.0;
      } else {
        r1 = r2 = d + half;
        i1 = std::sqrt(-disc);
        i2 = -i1;
      }
    }
    // first column of (H - s1 I)(H - s2 I) on the active block, scaled by
    // 1/sc and formed from the differences H(lo, lo) - s, which keeps it
    // accurate when the shifts lie close to the diagonal (a clustered
    // spectrum); the expanded polynomial would cancel there
    const double h00 = H[ix(lo, lo)], h10 = H[ix(lo + 1, lo)];
    const double sc = std::fabs(h00 - r2) + std::fabs(i2) + std::fabs(h10);
    const double h10s = sc > 0.0 ? h10 / sc : 0.0;
    double x = sc > 0.0 ? h10s * H[ix(lo, lo + 1)] + (h00 - r1) * ((h00 - r2) / sc) - i1 * (i2 / sc)
                        : 0.0;
    double y = h10s * (h00 + H[ix(lo + 1, lo + 1)] - r1 - r2);
    double z = h10s * H[ix(lo + 2, lo + 1)];
    for (int k = lo - 1; k + 3 <= hi; ++k) {
      // reflector on rows k+1..k+3 taking (x, y, z) to a multiple of e_1
      const double nrm = std::sqrt(x * x + y * y + z * z);
      if (nrm != 0.0) {
        double v[3] = {x + (x >= 0 ? nrm : -nrm), y, z};
        const double vn = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double f = 2.0 / vn;
        const int r0 = k + 1;
        refl_rows(v, 3, r0, std::max(lo, k), m, f);
        refl_cols(H, v, 3, r0, std::min(r0 + 4, hi + 1), f);
        refl_cols(Z, v, 3, r0, m, f);
        if (k >= lo) H[ix(k + 2, k)] = H[ix(k + 3, k)] = 0.0;
      }
      x = H[ix(k + 2, k + 1)];
      y = H[ix(k + 3, k + 1)];
      z = k + 4 <= hi ? H[ix(k + 4, k + 1)] : 0.0;
    }
    // last step: a rotation on rows hi-1, hi zeroing (x, y) -> (r, 0)
    {
      const double r = std::hypot(x, y);
      if (r != 0.0) {
        const int i = hi - 1;
        rot(i, x / r, y / r, std::max(lo, i - 1), hi + 1);
        if (i - 1 >= lo) H[ix(i + 1, i - 1)] = 0.0;
      }
    }
  }
  // complex Schur form: each remaining 2x2 block (a complex pair) made upper
  // triangular by U = [[x1, -conj x2], [x2, conj x1]], x a unit eigenvector
  t.assign(mm, cplx(0));
  q.assign(mm, cplx(0));
  for (size_t e = 0; e < mm; ++e) {
    t[e] = cplx(H[e], 0.0);
    q[e] = cplx(Z[e], 0.0);
  }
  for (int i = 0; i + 1 < m; ++i) {
    if (H[ix(i + 1, i)] == 0.0) continue;
    const double p = H[ix(i, i)], b = H[ix(i, i + 1)], c = H[ix(i + 1, i)], d = H[ix(i + 1, i + 1)];
    const double half = 0.5 * (p - d);
    const double disc = half * half + b * c;
    // disc < 0 here (real pairs were split); lambda = (p+d)/2 + i sqrt(-disc)
    const cplx lam(0.5 * (p + d), std::sqrt(std::max(-disc, 0.0)));
    // (B - lambda I) x = 0: x = (b, lambda - p)
    cplx x1(b, 0.0), x2 = lam - p;
    const double xn = std::sqrt(std::norm(x1) + std::norm(x2));
    x1 /= xn;
    x2 /= xn;
    const cplx u11 = x1, u21 = x2, u12 = -std::conj(x2), u22 = std::conj(x1);
    // rows i, i+1 <- U^H rows (columns i..m-1)
    for (int j = i; j < m; ++j) {
      const cplx r0 = t[ix(i, j)], r1 = t[ix(i + 1, j)];
      t[ix(i, j)] = std::conj(u11) * r0 + std::conj(u21) * r1;
      t[ix(i + 1, j)] = std::conj(u12) * r0 + std::conj(u22) * r1;
    }
    // columns i, i+1 <- columns U (rows 0..i+1 of T, all of Q)
    for (int which = 0; which < 2; ++which) {
      std::vector<cplx>& M = which ? q : t;
      const int n = which ? m : i + 2;
      for (int r = 0; r < n; ++r) {
        const cplx c0 = M[ix(r, i)], c1 = M[ix(r, i + 1)];
        M[ix(r, i)] = c0 * u11 + c1 * u21;
        M[ix(r, i + 1)] = c0 * u12 + c1 * u22;
      }
    }
    t[ix(i + 1, i)] = 0.0;
    ++i;  // the pair's second row is done
  }
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
