// Context, low-rank setup on the GPU (thick-restart Arnoldi), FGMRES and the
// C ABI declared in include/gemslr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>

#include "device.h"
#include "engine.h"

using gs::cplx;
using gs::Error;

struct gs_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  std::string err;
  int dtype = GS_F64;
  int precision = GS_PREC_F64;
  bool ready = false;
  gs_opts opts{};
  std::unique_ptr<gs::HostSetup<double>> hd;
  std::unique_ptr<gs::HostSetup<cplx>> hz;
  std::unique_ptr<gs::Engine> eng;
  // solve data: permuted A on the device and FGMRES work space
  std::unique_ptr<gs::DevMem> amem;
  int32_t* a_rp = nullptr;
  int32_t* a_ci = nullptr;
  void* a_v = nullptr;
  int32_t* perm = nullptr;
  std::unique_ptr<gs::DevMem> wmem;
  int w_m = -1;
  void* pin = nullptr;  // pinned staging for small device->host reads
  size_t pin_bytes = 0;
  hipEvent_t fg_ev[2] = {nullptr, nullptr};  // FGMRES: Hessenberg columns landed
  // per level: the exact W_l on the device while the engine holds it rounded
  // (narrower storage) and the host copy has not been fetched
  std::vector<std::unique_ptr<gs::DevMem>> wkeep;
  gs_info info{};
  std::vector<std::string> step_labels;  // of the last gs_apply_profile
  int nparts = 1;                         // of the last gs_setup (feature cut flags)
};

static std::string g_create_error;
// an error's message: on its context, or (calls without one: gs_create and
// the host stages) where gs_last_error(NULL) reads it
static void gs_set_err(gs_ctx* c, const char* m);

// Scratch region of gs_apply_noalloc: static device memory of the code
// object, one copy per GPU, so that entry point allocates nothing.  Host
// code never uses the symbol itself (on the host it is only a stand-in);
// gs_create resolves each device's address once with hipGetSymbolAddress,
// with that device current, and the apply takes that address.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on `device` (current), resolved on first use.
static hipError_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

namespace gs {

#define HIPCHK(x) hipcheck((x), #x)

template <class T> struct DevOf;
template <> struct DevOf<double> { using type = double; };
template <> struct DevOf<cplx> { using type = dcplx; };

static void* pinned(gs_ctx* c, size_t bytes) {
  if (bytes > c->pin_bytes) {
    if (c->pin) (void)hipHostFree(c->pin);
    c->pin = nullptr;
    HIPCHK(hipHostMalloc(&c->pin, bytes, hipHostMallocDefault));
    c->pin_bytes = bytes;
  }
  return c->pin;
}

template <class T> static HostSetup<T>& host(gs_ctx* c);
template <> HostSetup<double>& host<double>(gs_ctx* c) { return *c->hd; }
template <> HostSetup<cplx>& host<cplx>(gs_ctx* c) { return *c->hz; }

// ------------------------------------------------------------ small helpers
template <class DT> static DT from_host(double v);
template <> double from_host<double>(double v) { return v; }
template <> dcplx from_host<dcplx>(double v) { return mk(v, 0.0); }

// CGS with one re-orthogonalisation pass: w <- w - V (V^H w), twice; the
// coefficients of both passes are added into hacc (if not null).
template <class DT>
static void cgs2(const DT* V, int64_t ld, int ncol, DT* w, int64_t n, DT* partial, DT* h,
                 DT* hacc, hipStream_t st) {
  if (hacc) launch_fill<DT>(hacc, from_host<DT>(0.0), ncol, st);
  for (int pass = 0; pass < 2; ++pass) {
    launch_multidot<DT>(V, ld, ncol, w, n, partial, h, st);
    launch_gemv_sub<DT>(V, ld, ncol, h, w, n, hacc, st);
  }
}

// Schur form Sm = Q T Q^H (m x m) reordered so the k wanted Ritz values come
// first (k raised by one for a real matrix rather than split a pair); returns
// the basis G (m x kk) of the wanted invariant subspace and R = G^H Sm G:
// for complex data G = Q_k and R = T_k; for real data G is a real
// orthonormal basis of the conjugate-closed subspace (pivoted Gram-Schmidt on
// [Re Q_k, Im Q_k]) and R = G^T Sm G.
template <class T>
static int schur_basis_from(int m, const std::vector<cplx>& Sm, int k, std::vector<cplx>& Tm,
                            std::vector<cplx>& Q, std::vector<cplx>& theta_k, std::vector<T>& G,
                            std::vector<T>& R);

template <class T>
static int schur_basis(int m, const std::vector<cplx>& Sm, int k, std::vector<cplx>& Tm,
                       std::vector<cplx>& Q, std::vector<cplx>& theta_k, std::vector<T>& G,
                       std::vector<T>& R) {
  if (std::is_same<T, double>::value) {
    // real Rayleigh matrix: real double-shift iteration
    std::vector<double> Sr((size_t)m * m);
    for (size_t e = 0; e < Sr.size(); ++e) Sr[e] = Sm[e].real();
    schur_real(m, Sr, Tm, Q);
  } else {
    Tm = Sm;
    schur_complex(m, Tm, Q);
  }
  return schur_basis_from<T>(m, Sm, k, Tm, Q, theta_k, G, R);
}

// The same from a complex Schur form Tm = Q^H Sm Q already at hand (any
// order of the diagonal): reorder so the k wanted values lead, then G, R.
template <class T>
static int schur_basis_from(int m, const std::vector<cplx>& Sm, int k, std::vector<cplx>& Tm,
                            std::vector<cplx>& Q, std::vector<cplx>& theta_k, std::vector<T>& G,
                            std::vector<T>& R) {
  const bool real = std::is_same<T, double>::value;
  std::vector<cplx> theta(m);
  for (int i = 0; i < m; ++i) theta[i] = Tm[(size_t)i * m + i];
  std::vector<int> sel = select_wanted(theta, k, real);
  schur_reorder(m, Tm, Q, sel);
  int kk = 0;
  for (int x : sel) kk += x;
  theta_k.assign(kk, 0.0);
  for (int i = 0; i < kk; ++i) theta_k[i] = Tm[(size_t)i * m + i];
  G.assign((size_t)m * kk, T(0));
  R.assign((size_t)kk * kk, T(0));
  if (real) {
    std::vector<std::vector<double>> X;
    for (int j = 0; j < kk; ++j) {
      std::vector<double> re(m), im(m);
      for (int i = 0; i < m; ++i) { re[i] = Q[(size_t)j * m + i].real(); im[i] = Q[(size_t)j * m + i].imag(); }
      X.push_back(re);
      X.push_back(im);
    }
    double first = -1;
    double* g = (double*)G.data();
    for (int q = 0; q < kk; ++q) {
      int best = -1;
      double bn = -1;
      for (size_t x = 0; x < X.size(); ++x) {
        double nn2 = 0;
        for (double e : X[x]) nn2 += e * e;
        if (nn2 > bn) { bn = nn2; best = (int)x; }
      }
      bn = std::sqrt(bn);
      if (first < 0) first = bn;
      if (bn <= 1e-8 * first) throw Error(GS_EINVAL, "wanted Ritz set is not closed under conjugation");
      std::vector<double> qv = X[best];
      for (double& e : qv) e /= bn;
      X.erase(X.begin() + best);
      for (int pass = 0; pass < 2; ++pass)
        for (auto& x : X) {
          double d = 0;
          for (int i = 0; i < m; ++i) d += qv[i] * x[i];
          for (int i = 0; i < m; ++i) x[i] -= d * qv[i];
        }
      for (int i = 0; i < m; ++i) g[(size_t)q * m + i] = qv[i];
    }
    // R = G^T (Sm G): Sm G once (m x kk), then the kk x kk product
    double* r = (double*)R.data();
    std::vector<double> sg((size_t)m * kk, 0.0);
    for (int b = 0; b < kk; ++b)
      for (int j = 0; j < m; ++j) {
        const double gj = g[(size_t)b * m + j];
        if (gj == 0.0) continue;
        for (int i = 0; i < m; ++i) sg[(size_t)b * m + i] += Sm[(size_t)j * m + i].real() * gj;
      }
    for (int b = 0; b < kk; ++b)
      for (int a = 0; a < kk; ++a) {
        double acc = 0;
        for (int i = 0; i < m; ++i) acc += g[(size_t)a * m + i] * sg[(size_t)b * m + i];
        r[(size_t)b * kk + a] = acc;
      }
  } else {
    for (int j = 0; j < kk; ++j)
      for (int i = 0; i < m; ++i) std::memcpy((void*)&G[(size_t)j * m + i], &Q[(size_t)j * m + i], sizeof(cplx));
    for (int j = 0; j < kk; ++j)
      for (int i = 0; i < kk; ++i) std::memcpy((void*)&R[(size_t)j * kk + i], &Tm[(size_t)j * m + i], sizeof(cplx));
  }
  return kk;
}

template <class T> static cplx to_cplx(const void* p, size_t i);
template <> cplx to_cplx<double>(const void* p, size_t i) { return cplx(((const double*)p)[i], 0.0); }
template <> cplx to_cplx<cplx>(const void* p, size_t i) { return ((const cplx*)p)[i]; }

// ------------------------------------------------------------ low-rank setup
// Install W_l (device, s x k, value type) and the level's H_l in the engine,
// on the device.  The host copy of W_l is fetched only when the host needs
// it (fetch_host_w): from the engine when it stores W_l exactly, else from
// an exact device copy kept here.
template <class T>
static void install_lowrank(gs_ctx* c, int l, int k, const void* Wd) {
  HostLevel<T>& h = host<T>(c).lv[l];
  if (c->wkeep.size() <= (size_t)l) c->wkeep.resize((size_t)l + 1);
  c->wkeep[(size_t)l].reset();
  if (c->eng->set_lowrank_device(l, k, Wd, h.H.data()) == 0) {
    auto keep = std::make_unique<DevMem>();
    T* w = keep->alloc<T>((size_t)h.s * k);
    HIPCHK(hipMemcpyAsync(w, Wd, (size_t)h.s * k * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->wkeep[(size_t)l] = std::move(keep);
  }
  h.W.clear();
  h.W.shrink_to_fit();
  h.w_on_device = true;
}

// W_l of every level that only the engine holds, into the host setup
template <class T>
static void fetch_host_w(gs_ctx* c) {
  for (size_t l = 0; l < host<T>(c).lv.size(); ++l) {
    HostLevel<T>& h = host<T>(c).lv[l];
    if (!h.w_on_device) continue;
    h.W.resize((size_t)h.s * h.k);
    if (l < c->wkeep.size() && c->wkeep[l]) {
      HIPCHK(hipMemcpyAsync(h.W.data(), c->wkeep[l]->ptrs[0], h.W.size() * sizeof(T),
                            hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      c->wkeep[l].reset();
    } else if (!c->eng || !c->eng->get_lowrank_w((int)l, h.W.data())) {
      throw Error(GS_ESTATE, "W_l is held by no engine");
    }
    h.w_on_device = false;
  }
}
static void fetch_host_w_any(gs_ctx* c) {
  if (c->device >= 0) hipcheck(hipSetDevice(c->device), "hipSetDevice");
  if (c->dtype == GS_F64) {
    if (c->hd) fetch_host_w<double>(c);
  } else if (c->hz) {
    fetch_host_w<cplx>(c);
  }
}

// Thick-restart (Krylov-Schur) Arnoldi on Ĝ_l on the GPU (Sec. 2.3, Sec. 4.2):
// cycle length m = 2k, Ritz pairs accepted when |b^H y| <= tol |theta|.
// Orthogonalisation and the basis are float64 / complex128 whatever the
// storage precision of the factors used inside Ĝ_l.
template <class T>
static void lowrank_level(gs_ctx* c, int l, int kreq, const float* Ystart = nullptr) {
  using DT = typename DevOf<T>::type;
  const bool real = std::is_same<T, double>::value;
  HostSetup<T>& S = host<T>(c);
  HostLevel<T>& h = S.lv[l];
  const hipStream_t st = c->stream;
  const int64_t s = h.s;
  const int k = (int)std::min<int64_t>(kreq, s);
  if (k <= 0) return;
  int m = (int)std::min<int64_t>(2 * (int64_t)k, s);
  if (m <= k) m = (int)std::min<int64_t>(k + 1, s);
  DevMem mem;
  DT* V = mem.alloc<DT>((size_t)s * (m + 1));
  DT* w = mem.alloc<DT>(s);
  DT* tmp = mem.alloc<DT>((size_t)s * (m + 1));
  DT* hd = mem.alloc<DT>(m + 1);
  DT* hacc = mem.alloc<DT>(m + 1);
  DT* part = mem.alloc<DT>((size_t)256 * (m + 1));
  double* npart = mem.alloc<double>(256);
  double* nrm = mem.alloc<double>(2);
  DT* Gd = mem.alloc<DT>((size_t)m * m);
  std::vector<DT> hv(s);
  std::vector<double> v0(s);
  auto upload_start = [&](uint64_t sd, DT* dst) {
    start_vector(sd, s, v0.data());
    for (int64_t i = 0; i < s; ++i) hv[i] = from_host<DT>(v0[i]);
    HIPCHK(hipMemcpyAsync(dst, hv.data(), s * sizeof(DT), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  const uint64_t seed = c->opts.seed + (uint64_t)l;
  upload_start(seed, V);
  if (Ystart) {
    // a start vector in the predicted subspace: v_0 = Y (Y^T r), Y the
    // starting basis (s x k, row-major float32, device)
    DT* Yc = tmp;  // s x k, column-major
    launch_rows_to_cols<DT>(Ystart, s, k, kreq, Yc, s, st);
    launch_multidot<DT>(Yc, s, k, V, s, part, hd, st);
    launch_copy<DT>(V, w, s, st);
    launch_fill<DT>(V, from_host<DT>(0.0), s, st);
    launch_gemv_add<DT>(Yc, s, k, hd, V, s, st);
  }
  launch_norm<DT>(V, s, npart, nrm, st);
  launch_scale_inv<DT>(V, nrm, V, s, st);

  std::vector<cplx> Sm((size_t)(m + 1) * m, cplx(0));  // Krylov decomposition G V = V S
  auto Sat = [&](int i, int j) -> cplx& { return Sm[(size_t)j * (m + 1) + i]; };
  const size_t stage_bytes = (m + 1) * sizeof(DT) + 2 * sizeof(double);
  // device copy of the cycle's Hessenberg columns and norms, read once per
  // cycle instead of once per step
  DT* Sd = mem.alloc<DT>((size_t)(m + 1) * m);
  double* nd = mem.alloc<double>((size_t)2 * m + 1);  // + breakdown flag
  std::vector<DT> Sh((size_t)(m + 1) * m);
  std::vector<double> nh((size_t)2 * m + 1);
  // nmv: products of the Krylov decomposition (it also salts the fresh start
  // directions after a breakdown); redone: products of cycles that broke
  // down, computed and discarded before the step-by-step rerun
  int j0 = 0, nmv = 0, redone = 0;
  const int maxcyc = std::max(1, c->opts.arnoldi_max_cycles);
  for (int cycle = 0; cycle < maxcyc; ++cycle) {
    // steps j0..m-1 without host round trips; a breakdown (flagged by the
    // device) sends the cycle through the step-by-step path below
    bool stepwise = false;
    {
      launch_fill<double>(nd + 2 * m, 0.0, 1, st);
      for (int j = j0; j < m; ++j) {
        c->eng->ghat(l, V + (size_t)j * s, w);
        launch_norm<DT>(w, s, npart, nrm + 1, st);
        cgs2<DT>(V, s, j + 1, w, s, part, hd, hacc, st);
        launch_norm<DT>(w, s, npart, nrm, st);
        launch_arnoldi_step<DT>(hacc, j + 1, nrm, Sd + (size_t)j * (m + 1), nd + 2 * j, nd + 2 * m,
                                w, V + (size_t)(j + 1) * s, s, st);
      }
      HIPCHK(hipMemcpyAsync(Sh.data(), Sd, Sh.size() * sizeof(DT), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(nh.data(), nd, nh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (nh[2 * m] != 0.0) {
        stepwise = true;  // redo from j0: column j0 of V is untouched
        redone += m - j0;
      } else {
        nmv += m - j0;
        for (int j = j0; j < m; ++j) {
          for (int i = 0; i <= j; ++i) {
            cplx v;
            if (real) v = cplx(((const double*)Sh.data())[(size_t)j * (m + 1) + i], 0.0);
            else std::memcpy((void*)&v, &Sh[(size_t)j * (m + 1) + i], sizeof(DT));
            Sat(i, j) = v;
          }
          Sat(j + 1, j) = nh[2 * j];
        }
      }
    }
    for (int j = j0; stepwise && j < m; ++j) {
      c->eng->ghat(l, V + (size_t)j * s, w);
      ++nmv;
      launch_norm<DT>(w, s, npart, nrm + 1, st);
      cgs2<DT>(V, s, j + 1, w, s, part, hd, hacc, st);
      launch_norm<DT>(w, s, npart, nrm, st);
      char* pb = (char*)pinned(c, stage_bytes);
      HIPCHK(hipMemcpyAsync(pb, hacc, (j + 1) * sizeof(DT), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(pb + (m + 1) * sizeof(DT), nrm, 2 * sizeof(double),
                            hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      const DT* hh = (const DT*)pb;
      const double* nn = (const double*)(pb + (m + 1) * sizeof(DT));
      for (int i = 0; i <= j; ++i) {
        cplx v;
        std::memcpy((void*)&v, &hh[i], sizeof(DT));
        if (real) v = cplx(((const double*)hh)[i], 0.0);
        Sat(i, j) = v;
      }
      const double beta = nn[0], wn = nn[1];
      DT* vnext = V + (size_t)(j + 1) * s;
      if (beta > 1e-12 * wn) {
        Sat(j + 1, j) = beta;
        launch_scale_inv<DT>(w, nrm, vnext, s, st);
      } else {
        Sat(j + 1, j) = 0.0;
        if (j + 1 < m) {
          upload_start(c->opts.seed + (uint64_t)l + 0x5DEECE66DULL * (uint64_t)nmv, vnext);
          cgs2<DT>(V, s, j + 1, vnext, s, part, hd, nullptr, st);
          launch_norm<DT>(vnext, s, npart, nrm, st);
          launch_scale_inv<DT>(vnext, nrm, vnext, s, st);
        } else {
          launch_fill<DT>(vnext, from_host<DT>(0.0), s, st);
        }
      }
    }
    // Schur form of the m x m Rayleigh matrix, wanted values first
    std::vector<cplx> Sorig((size_t)m * m), Tm, Q, thk;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) Sorig[(size_t)j * m + i] = Sat(i, j);
    std::vector<T> G, R;
    const int kk = schur_basis<T>(m, Sorig, k, Tm, Q, thk, G, R);
    // residuals of the wanted Ritz pairs: |b Q_k y_i|
    std::vector<cplx> Tk((size_t)kk * kk), Y;
    for (int j = 0; j < kk; ++j)
      for (int i = 0; i < kk; ++i) Tk[(size_t)j * kk + i] = Tm[(size_t)j * m + i];
    triu_eigvecs(kk, Tk, Y);
    std::vector<cplx> bq(kk, 0.0);
    for (int j = 0; j < kk; ++j)
      for (int i = 0; i < m; ++i) bq[j] += Sat(m, i) * Q[(size_t)j * m + i];
    bool conv = true;
    for (int i = 0; i < kk; ++i) {
      cplx r = 0;
      for (int j = 0; j < kk; ++j) r += bq[j] * Y[(size_t)i * kk + j];
      if (std::abs(r) > c->opts.arnoldi_tol * std::abs(thk[i])) conv = false;
    }
    HIPCHK(hipMemcpyAsync(Gd, G.data(), G.size() * sizeof(DT), hipMemcpyHostToDevice, st));
    const bool last = conv || cycle == maxcyc - 1 || kk >= m;
    if (last) {
      launch_gemm_small<DT>(V, s, m, Gd, kk, tmp, s, s, st);
      h.k = kk;
      h.H = correction_matrix<T>(kk, R, thk);
      h.arnoldi_cycles = cycle + 1;
      h.arnoldi_matvecs = nmv + redone;
      h.arnoldi_converged = conv ? 1 : 0;
      install_lowrank<T>(c, l, kk, tmp);
      return;
    }
    // thick restart: V[:, :kk] = V_m G, V[:, kk] = v_{m+1}
    launch_gemm_small<DT>(V, s, m, Gd, kk, tmp, s, s, st);
    launch_copy<DT>(tmp, V, (int64_t)s * kk, st);
    launch_copy<DT>(V + (size_t)m * s, V + (size_t)kk * s, s, st);
    HIPCHK(hipStreamSynchronize(st));
    std::vector<cplx> bg(kk, 0.0);
    for (int j = 0; j < kk; ++j)
      for (int i = 0; i < m; ++i) {
        cplx gij;
        if (real) gij = cplx(((double*)G.data())[(size_t)j * m + i], 0);
        else std::memcpy((void*)&gij, &G[(size_t)j * m + i], sizeof(cplx));
        bg[j] += Sat(m, i) * gij;
      }
    std::fill(Sm.begin(), Sm.end(), cplx(0));
    for (int j = 0; j < kk; ++j)
      for (int i = 0; i < kk; ++i) {
        cplx r;
        if (real) r = cplx(((double*)R.data())[(size_t)j * kk + i], 0);
        else std::memcpy((void*)&r, &R[(size_t)j * kk + i], sizeof(cplx));
        Sat(i, j) = r;
      }
    for (int j = 0; j < kk; ++j) Sat(kk, j) = bg[j];
    j0 = kk;
  }
}


// Block Rayleigh-Ritz iteration from a given starting basis Y (s x k, row-major
// float32, device).  The search space V (orthonormal, at most mmax = 3k
// columns) starts as orth(Y).  Each iteration takes the Ritz pairs of
// T = V^H G V for the k wanted values, accepts when every pair has
// ||G x - theta x|| <= tol |theta|, and otherwise adds the residuals of the
// pairs not yet accepted (accepted pairs cost no further products); when the
// space would exceed mmax it is first truncated to the leading wanted Ritz
// vectors (a thick restart).  T and M = (G V)^H (G V) are kept up to date
// column by column, so each residual norm is sqrt(y^H M y - |theta|^2) for
// the unit coefficient vector y, with no pass over the residual block.
// Returns true and installs W_l, H_l on acceptance; fails once the products
// reach block_max_iters * k (the caller then runs the restarted Arnoldi).
template <class T>
static bool lowrank_block(gs_ctx* c, int l, int kreq, const float* Y) {
  using DT = typename DevOf<T>::type;
  const bool real = std::is_same<T, double>::value;
  HostSetup<T>& S = host<T>(c);
  HostLevel<T>& h = S.lv[l];
  const hipStream_t st = c->stream;
  const int64_t s = h.s;
  const int k = (int)std::min<int64_t>(kreq, s);
  if (k <= 0) return true;
  const int mmax = (int)std::min<int64_t>(std::max(3 * k, k + 8), s);
  const int cap = mmax + 2;           // a kept conjugate pair may add one
  const int bmax = 2 * k + 2;         // staged expansion columns
  DevMem mem;
  DT* Sv = mem.alloc<DT>((size_t)s * cap);   // V
  DT* GSv = mem.alloc<DT>((size_t)s * cap);  // G V
  DT* X = mem.alloc<DT>((size_t)s * bmax);   // staged new directions
  DT* tmp = mem.alloc<DT>((size_t)s * std::max(cap, bmax));
  DT* part = mem.alloc<DT>((size_t)256 * cap);
  DT* hd = mem.alloc<DT>(cap);
  DT* Td = mem.alloc<DT>((size_t)cap * cap);  // dots, column-major, ld cap
  DT* Md = mem.alloc<DT>((size_t)cap * cap);
  DT* Cd = mem.alloc<DT>((size_t)cap * std::max(cap, bmax));  // small coefficient blocks
  double* npart = mem.alloc<double>(256);
  double* nrm = mem.alloc<double>(2);
  std::vector<DT> hv(s);
  std::vector<double> v0(s);
  std::vector<cplx> Th((size_t)cap * cap, 0.0), Mh((size_t)cap * cap, 0.0);
  auto col = [&](DT* base, int j) { return base + (size_t)j * s; };
  auto at = [&](std::vector<cplx>& A, int i, int j) -> cplx& { return A[(size_t)j * cap + i]; };
  int w = 0, nmv = 0, fresh = 0;
  const int budget = std::max(1, c->opts.block_max_iters) * k;

  auto upload = [&](const std::vector<cplx>& A, int r, int cc, DT* dst) {
    std::vector<DT> t((size_t)r * cc);
    for (size_t i = 0; i < t.size(); ++i) {
      if (real) ((double*)t.data())[i] = A[i].real();
      else std::memcpy((void*)&t[i], &A[i], sizeof(cplx));
    }
    HIPCHK(hipMemcpyAsync(dst, t.data(), t.size() * sizeof(DT), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  // append column src to V if it keeps a relative norm > 1e-6 after two
  // Gram-Schmidt passes against V; its product with G is formed by flush,
  // for all columns appended since the last flush in one batched product
  int wg = 0;  // columns of V whose products G V are formed
  auto flush = [&]() {
    if (w > wg) {
      c->eng->ghat_batch(l, w - wg, col(Sv, wg), col(GSv, wg));
      nmv += w - wg;
      wg = w;
    }
  };
  auto append = [&](const DT* src) -> bool {
    launch_copy<DT>(src, col(Sv, w), s, st);
    launch_norm<DT>(col(Sv, w), s, npart, nrm + 1, st);
    if (w > 0) cgs2<DT>(Sv, s, w, col(Sv, w), s, part, hd, nullptr, st);
    launch_norm<DT>(col(Sv, w), s, npart, nrm, st);
    double nn[2];
    HIPCHK(hipMemcpyAsync(nn, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (!(nn[0] > 1e-6 * nn[1] && nn[0] > 0)) return false;
    launch_scale_inv<DT>(col(Sv, w), nrm, col(Sv, w), s, st);
    ++w;
    return true;
  };
  // T and M entries that involve the columns [w0, w)
  auto extend_dots = [&](int w0) {
    flush();
    if (w0 == w) return;
    for (int j = w0; j < w; ++j) {
      launch_multidot<DT>(Sv, s, w, col(GSv, j), s, part, Td + (size_t)j * cap, st);
      launch_multidot<DT>(GSv, s, w, col(GSv, j), s, part, Md + (size_t)j * cap, st);
    }
    // T[i, j] for a new column i and an old column j is conj((G v_j)^H v_i):
    // one multi-dot per new column against the old products (staged in Cd)
    // instead of one per old column
    for (int i = w0; i < w; ++i)
      launch_multidot<DT>(GSv, s, w0, col(Sv, i), s, part, Cd + (size_t)(i - w0) * cap, st);
    std::vector<DT> tt((size_t)cap * cap), mm((size_t)cap * cap), tn((size_t)cap * (w - w0));
    HIPCHK(hipMemcpyAsync(tn.data(), Cd, tn.size() * sizeof(DT), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(tt.data(), Td, tt.size() * sizeof(DT), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(mm.data(), Md, mm.size() * sizeof(DT), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int j = w0; j < w; ++j)
      for (int i = 0; i < w; ++i) {
        at(Th, i, j) = to_cplx<T>(tt.data(), (size_t)j * cap + i);
        at(Mh, i, j) = to_cplx<T>(mm.data(), (size_t)j * cap + i);
        at(Mh, j, i) = std::conj(at(Mh, i, j));
      }
    for (int i = 0; i < w0; ++i)
      for (int j = w0; j < w; ++j)
        at(Th, j, i) = std::conj(to_cplx<T>(tn.data(), (size_t)(j - w0) * cap + i));
  };
  auto square = [&](const std::vector<cplx>& A, int m) {
    std::vector<cplx> B((size_t)m * m);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) B[(size_t)j * m + i] = A[(size_t)j * cap + i];
    return B;
  };
  auto as_cplx = [&](const std::vector<T>& G) {
    std::vector<cplx> out(G.size());
    for (size_t i = 0; i < G.size(); ++i) out[i] = to_cplx<T>(G.data(), i);
    return out;
  };

  // initial space: the columns of Y, topped up with generator vectors
  launch_rows_to_cols<DT>(Y, s, k, kreq, X, s, st);
  for (int j = 0; j < k; ++j) append(col(X, j));
  while (w < k) {
    if (fresh > 4 * k) throw Error(GS_EINVAL, "could not build the block basis");
    start_vector(c->opts.seed + (uint64_t)l + 0x9E3779B9ULL * (uint64_t)(++fresh), s, v0.data());
    for (int64_t i = 0; i < s; ++i) hv[i] = from_host<DT>(v0[i]);
    HIPCHK(hipMemcpyAsync(X, hv.data(), s * sizeof(DT), hipMemcpyHostToDevice, st));
    append(X);
  }
  extend_dots(0);
  for (int it = 0;; ++it) {
    const std::vector<cplx> Tw = square(Th, w);
    std::vector<cplx> Tm, Q, thk;
    std::vector<T> G, R;
    const int kk = schur_basis<T>(w, Tw, k, Tm, Q, thk, G, R);
    std::vector<cplx> Tk((size_t)kk * kk), Ye;
    for (int j = 0; j < kk; ++j)
      for (int i = 0; i < kk; ++i) Tk[(size_t)j * kk + i] = Tm[(size_t)j * w + i];
    triu_eigvecs(kk, Tk, Ye);
    // unit coefficient vectors y_e = Q_k Ye[:, e] and their residual norms
    std::vector<std::vector<cplx>> todo;
    for (int e = 0; e < kk; ++e) {
      std::vector<cplx> y(w, 0.0);
      for (int j = 0; j < kk; ++j)
        for (int i = 0; i < w; ++i) y[i] += Q[(size_t)j * w + i] * Ye[(size_t)e * kk + j];
      double yn = 0;
      for (const cplx& v : y) yn += std::norm(v);
      yn = std::sqrt(yn);
      for (cplx& v : y) v /= yn;
      cplx q = 0;
      for (int b = 0; b < w; ++b) {
        cplx mb = 0;
        for (int a = 0; a < w; ++a) mb += std::conj(y[a]) * at(Mh, a, b);
        q += mb * y[b];
      }
      const double res2 = q.real() - std::norm(thk[e]);
      if (std::sqrt(std::max(0.0, res2)) <= c->opts.arnoldi_tol * std::abs(thk[e])) continue;
      if (real && thk[e].imag() < -1e-10 * std::abs(thk[e])) continue;  // partner of a pair
      todo.push_back(y);
    }
    if (todo.empty()) {
      upload(as_cplx(G), w, kk, Cd);
      launch_gemm_small<DT>(Sv, s, w, Cd, kk, tmp, s, s, st);
      h.k = kk;
      h.H = correction_matrix<T>(kk, R, thk);
      h.arnoldi_cycles = it + 1;
      h.arnoldi_matvecs = nmv;
      h.arnoldi_converged = 1;
      install_lowrank<T>(c, l, kk, tmp);
      return true;
    }
    if (nmv >= budget) break;
    // coefficient block P (w x nb): y_e, or for real data Re y_e and Im y_e
    // (a real eigenvalue's vector is rotated to be real first)
    std::vector<cplx> P;
    int nb = 0;
    for (std::vector<cplx>& y : todo) {
      if (real) {
        size_t big = 0;
        for (size_t i = 1; i < y.size(); ++i)
          if (std::abs(y[i]) > std::abs(y[big])) big = i;
        const cplx ph = std::abs(y[big]) > 0 ? std::conj(y[big]) / std::abs(y[big]) : cplx(1.0);
        for (cplx& v : y) v *= ph;
        for (int part_im = 0; part_im < 2 && nb < bmax; ++part_im) {
          double pn = 0;
          for (const cplx& v : y) pn += part_im ? v.imag() * v.imag() : v.real() * v.real();
          if (part_im && pn <= 1e-20) break;
          for (const cplx& v : y) P.push_back(part_im ? v.imag() : v.real());
          ++nb;
        }
      } else if (nb < bmax) {
        P.insert(P.end(), y.begin(), y.end());
        ++nb;
      }
    }
    // X = (G V) P - V (T P): the residual block of the chosen vectors
    std::vector<cplx> TP((size_t)w * nb, 0.0);
    for (int j = 0; j < nb; ++j)
      for (int a = 0; a < w; ++a) {
        const cplx pa = P[(size_t)j * w + a];
        for (int i = 0; i < w; ++i) TP[(size_t)j * w + i] += Tw[(size_t)a * w + i] * pa;
      }
    upload(P, w, nb, Cd);
    launch_gemm_small<DT>(GSv, s, w, Cd, nb, X, s, s, st);
    upload(TP, w, nb, Cd);
    launch_gemm_small<DT>(Sv, s, w, Cd, nb, tmp, s, s, st);
    launch_sub<DT>(X, tmp, X, (int64_t)s * nb, st);
    // thick restart to the leading wanted Ritz vectors when the space is full
    if (w + nb > mmax) {
      const int keep = std::max(k, mmax - nb);
      if (keep < w) {
        // the Schur form of T from this iteration, reordered for `keep`
        std::vector<cplx> Tm2 = Tm, Q2 = Q, th2;
        std::vector<T> G2, R2;
        const int k2 = schur_basis_from<T>(w, Tw, keep, Tm2, Q2, th2, G2, R2);
        const std::vector<cplx> Gc = as_cplx(G2);
        upload(Gc, w, k2, Cd);
        launch_gemm_small<DT>(Sv, s, w, Cd, k2, tmp, s, s, st);
        launch_copy<DT>(tmp, Sv, (int64_t)s * k2, st);
        launch_gemm_small<DT>(GSv, s, w, Cd, k2, tmp, s, s, st);
        launch_copy<DT>(tmp, GSv, (int64_t)s * k2, st);
        // T <- G^H T G, M <- G^H M G
        std::vector<cplx> T2((size_t)cap * cap, 0.0), M2((size_t)cap * cap, 0.0);
        for (int pass = 0; pass < 2; ++pass) {
          std::vector<cplx>& A = pass ? Mh : Th;
          std::vector<cplx>& B = pass ? M2 : T2;
          std::vector<cplx> AG((size_t)w * k2, 0.0);
          for (int j = 0; j < k2; ++j)
            for (int a = 0; a < w; ++a) {
              const cplx g = Gc[(size_t)j * w + a];
              for (int i = 0; i < w; ++i) AG[(size_t)j * w + i] += at(A, i, a) * g;
            }
          for (int j = 0; j < k2; ++j)
            for (int i = 0; i < k2; ++i) {
              cplx v = 0;
              for (int a = 0; a < w; ++a) v += std::conj(Gc[(size_t)i * w + a]) * AG[(size_t)j * w + a];
              B[(size_t)j * cap + i] = v;
            }
          A.swap(B);
        }
        w = k2;
        wg = w;
      }
    }
    const int w0 = w;
    for (int j = 0; j < nb && w < cap; ++j) append(col(X, j));
    if (w == w0) break;  // no new direction survived: stagnation
    extend_dots(w0);
  }
  h.arnoldi_matvecs = nmv;
  return false;
}

// ------------------------------------------------------------ FGMRES
template <class T>
static int fgmres(gs_ctx* c, const void* b_user, void* x_user, double tol, gs_info* info) {
  using DT = typename DevOf<T>::type;
  const hipStream_t st = c->stream;
  const int64_t n = host<T>(c).n;
  const int m = std::max(1, c->opts.fgmres_restart);
  const int maxit = std::max(1, c->opts.maxit);
  const double t0 = now_s();
  if (c->w_m != m || !c->wmem) {
    c->wmem.reset();
    c->wmem = std::make_unique<DevMem>();
    c->w_m = m;
  }
  DevMem& M = *c->wmem;
  if (M.ptrs.empty()) {
    M.alloc<DT>((size_t)n * (m + 1));  // V
    M.alloc<DT>((size_t)n * m);        // Z
    M.alloc<DT>(n);                    // w
    M.alloc<DT>(n);                    // r
    M.alloc<DT>(n);                    // xp
    M.alloc<DT>(n);                    // bp
    M.alloc<DT>(m + 1);                // h
    M.alloc<DT>(m + 1);                // hacc
    M.alloc<DT>((size_t)256 * (m + 1));// partial
    M.alloc<double>(256);              // norm partials
    M.alloc<double>(4);                // norms
  }
  DT* V = (DT*)M.ptrs[0];
  DT* Z = (DT*)M.ptrs[1];
  DT* w = (DT*)M.ptrs[2];
  DT* r = (DT*)M.ptrs[3];
  DT* xp = (DT*)M.ptrs[4];
  DT* bp = (DT*)M.ptrs[5];
  DT* hd = (DT*)M.ptrs[6];
  DT* hacc = (DT*)M.ptrs[7];
  DT* part = (DT*)M.ptrs[8];
  double* npart = (double*)M.ptrs[9];
  double* nrm = (double*)M.ptrs[10];
  launch_permute<DT>((const DT*)b_user, c->perm, bp, n, false, st);
  launch_permute<DT>((const DT*)x_user, c->perm, xp, n, false, st);
  const DT* Av = (const DT*)c->a_v;
  auto read_norm = [&]() {
    double* pb = (double*)pinned(c, 64);
    HIPCHK(hipMemcpyAsync(pb, nrm, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return pb[0];
  };
  launch_norm<DT>(bp, n, npart, nrm, st);
  const double nb = read_norm();
  int its = 0;
  double relres = 0;
  bool converged = false;
  std::vector<T> Hh((size_t)(m + 1) * m), g(m + 1), sn(m), y(m);
  std::vector<double> cs(m);
  auto H_ = [&](int i, int j) -> T& { return Hh[(size_t)j * (m + 1) + i]; };
  if (nb == 0) {
    launch_fill<DT>(xp, from_host<DT>(0.0), n, st);
    converged = true;
  }
  while (!converged) {
    launch_residual<DT>(c->a_rp, c->a_ci, Av, xp, bp, r, n, st);
    launch_norm<DT>(r, n, npart, nrm, st);
    const double beta = read_norm();
    relres = beta / nb;
    if (relres <= tol) { converged = true; break; }
    if (its >= maxit) break;
    launch_scale_inv<DT>(r, nrm, V, n, st);
    std::fill(Hh.begin(), Hh.end(), T(0));
    std::fill(g.begin(), g.end(), T(0));
    g[0] = beta;
    int jend = 0;
    // Step j's device work (apply, product, orthogonalisation, next basis
    // vector) needs nothing from the host, which only turns the Hessenberg
    // columns into Givens rotations for the residual estimate and the final
    // least-squares solve.  So step j + 1 is queued before the host waits
    // for column j: the device never waits for the host.  A step queued
    // after the one that ends the cycle is left unused (its columns are
    // past jend).  Columns land in two pinned slots, step j's in slot j % 2.
    const size_t slot = ((size_t)(m + 1) * sizeof(DT) + sizeof(double) + 15) & ~(size_t)15;
    char* pslots = (char*)pinned(c, 2 * slot);
    auto issue = [&](int j) {
      c->eng->apply(V + (size_t)j * n, Z + (size_t)j * n, true);
      launch_spmv<DT>(c->a_rp, c->a_ci, Av, Z + (size_t)j * n, w, n, st);
      cgs2<DT>(V, n, j + 1, w, n, part, hd, hacc, st);
      launch_norm<DT>(w, n, npart, nrm, st);
      launch_scale_inv<DT>(w, nrm, V + (size_t)(j + 1) * n, n, st);
      char* pb = pslots + (size_t)(j % 2) * slot;
      HIPCHK(hipMemcpyAsync(pb, hacc, (j + 1) * sizeof(DT), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(pb + (m + 1) * sizeof(DT), nrm, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipEventRecord(c->fg_ev[j % 2], st));
    };
    for (hipEvent_t& e : c->fg_ev)
      if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    issue(0);
    for (int j = 0; j < m; ++j) {
      // its counts the steps finished before this one
      if (j + 1 < m && its + 1 < maxit) issue(j + 1);
      HIPCHK(hipEventSynchronize(c->fg_ev[j % 2]));
      const char* pb = pslots + (size_t)(j % 2) * slot;
      for (int i = 0; i <= j; ++i) std::memcpy((void*)&H_(i, j), pb + i * sizeof(DT), sizeof(DT));
      double hn;
      std::memcpy(&hn, pb + (m + 1) * sizeof(DT), sizeof(double));
      H_(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {
        T t1 = cs[i] * H_(i, j) + sn[i] * H_(i + 1, j);
        T t2 = -conjv(sn[i]) * H_(i, j) + cs[i] * H_(i + 1, j);
        H_(i, j) = t1;
        H_(i + 1, j) = t2;
      }
      // Givens rotation G = [[c, s], [-conj s, c]], c real, zeroing H(j+1, j)
      const T a = H_(j, j), bb = H_(j + 1, j);
      double cc;
      T ss, rr;
      if (absval(bb) == 0) { cc = 1; ss = T(0); rr = a; }
      else if (absval(a) == 0) { cc = 0; ss = conjv(bb) / absval(bb); rr = T(absval(bb)); }
      else {
        const double tt = std::hypot(absval(a), absval(bb));
        const T ph = a / absval(a);
        cc = absval(a) / tt;
        ss = ph * conjv(bb) / tt;
        rr = ph * tt;
      }
      cs[j] = cc;
      sn[j] = ss;
      H_(j, j) = rr;
      H_(j + 1, j) = T(0);
      g[j + 1] = -conjv(ss) * g[j];
      g[j] = cc * g[j];
      ++its;
      jend = j + 1;
      if (absval(g[j + 1]) <= tol * nb || its >= maxit || hn == 0) break;
    }
    for (int i = jend - 1; i >= 0; --i) {
      T sacc = g[i];
      for (int q = i + 1; q < jend; ++q) sacc -= H_(i, q) * y[q];
      y[i] = sacc / H_(i, i);
    }
    HIPCHK(hipMemcpyAsync(hd, y.data(), jend * sizeof(DT), hipMemcpyHostToDevice, st));
    launch_gemv_add<DT>(Z, n, jend, hd, xp, n, st);
    HIPCHK(hipStreamSynchronize(st));
  }
  launch_permute<DT>(xp, c->perm, (DT*)x_user, n, true, st);
  HIPCHK(hipStreamSynchronize(st));
  c->info.its = its;
  c->info.relres = relres;
  c->info.converged = converged ? 1 : 0;
  c->info.t_solve = now_s() - t0;
  if (info) *info = c->info;
  return converged ? GS_OK : GS_NOT_CONVERGED;
}

// ------------------------------------------------------------ setup helpers
template <class T>
static void host_stats(gs_ctx* c) {
  HostSetup<T>& S = host<T>(c);
  gs_info& I = c->info;
  I.nlevels = S.L();
  I.nnz_lu = 0;
  I.nnz_ef = 0;
  I.nnz_a = S.A.nnz();
  double lr = 0;
  for (int l = 0; l <= S.L() && l <= GS_MAX_LEVELS; ++l) {
    const HostLevel<T>& h = S.lv[l];
    I.d[l] = h.d;
    I.s[l] = h.s;
    I.nblocks[l] = (int64_t)h.blocks.size() - 1;
    I.k[l] = h.k;
    I.arnoldi_cycles[l] = h.arnoldi_cycles;
    I.arnoldi_matvecs[l] = h.arnoldi_matvecs;
    I.arnoldi_converged[l] = h.arnoldi_converged;
    I.nnz_lu += h.L.nnz() + h.U.nnz();
    I.nnz_ef += h.E.nnz() + h.F.nnz();
    lr += (double)h.s * h.k + (double)h.k * h.k;
  }
  I.fill = (double)I.nnz_lu / (double)std::max<int64_t>(1, I.nnz_a);
  I.fill_lowrank = ((double)I.nnz_lu + lr) / (double)std::max<int64_t>(1, I.nnz_a);
}

template <class T>
static void finish_setup(gs_ctx* c) {
  HostSetup<T>& S = host<T>(c);
  using DT = typename DevOf<T>::type;
  if (c->device < 0) {
    // host-only context: the host copy only (export, inspection)
    host_stats<T>(c);
    c->ready = true;
    return;
  }
  // permuted A for the solver
  c->amem = std::make_unique<DevMem>();
  const CSR<T>& Ap = S.Ap;
  std::vector<int32_t> rp(Ap.rp.begin(), Ap.rp.end());
  std::vector<int32_t> p32(S.perm.begin(), S.perm.end());
  c->a_rp = c->amem->alloc<int32_t>(rp.size());
  c->a_ci = c->amem->alloc<int32_t>(Ap.ci.size());
  c->a_v = c->amem->alloc<DT>(Ap.v.size());
  c->perm = c->amem->alloc<int32_t>(p32.size());
  HIPCHK(hipMemcpyAsync(c->a_rp, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->a_ci, Ap.ci.data(), Ap.ci.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->a_v, Ap.v.data(), Ap.v.size() * sizeof(DT), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->perm, p32.data(), p32.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->wmem.reset();
  c->w_m = -1;
  host_stats<T>(c);
  gs_info& I = c->info;
  c->eng->stats(&I, 0);
  I.apply_bytes = c->eng->bytes_per_apply();
  c->ready = true;
}

template <class T>
static void copy_csr(int64_t nr, int64_t nc, const int64_t* rp, const int32_t* ci, const void* v,
                     CSR<T>& out) {
  out = CSR<T>();
  out.nrows = nr;
  out.ncols = nc;
  out.rp.assign(rp, rp + nr + 1);
  const int64_t nnz = rp[nr];
  out.ci.assign(ci, ci + nnz);
  out.v.resize(nnz);
  if (nnz) std::memcpy((void*)out.v.data(), v, nnz * sizeof(T));
}

// the low-rank kernels take k <= 1024 per level (k = min(rank, s_l)); checked
// before any factorisation or Arnoldi work
template <class T>
static void check_rank(const HostSetup<T>& S, int rank) {
  for (int l = 0; l < S.L(); ++l)
    if (std::min<int64_t>(rank, S.lv[l].s) > 1024)
      throw Error(GS_EINVAL, "rank above 1024 on level " + std::to_string(l) +
                                 " is not supported");
}

static inline void set_imag_shift(double& s, double v) { (void)v; s = 0.0; }
static inline void set_imag_shift(cplx& s, double v) { s = cplx(0.0, v); }

template <class T>
static void setup_native(gs_ctx* c, int64_t n, const int64_t* rp, const int32_t* ci,
                         const void* val, int levels, int nparts, int rank, double drop_tol) {
  auto S = std::make_unique<HostSetup<T>>();
  copy_csr<T>(n, n, rp, ci, val, S->A);
  double t0 = now_s();
  // the caller's partition, else the geometric separator for grid
  // operators and nested dissection otherwise
  Partition part =
      c->opts.part_perm
          ? user_partition(n, rp, ci, c->opts.part_perm, c->opts.part_level_start,
                           c->opts.part_nlevels, c->opts.part_block_ptr, c->opts.part_block_count)
      : c->opts.grid_ndim > 0
          ? partition_grid(c->opts.grid_ndim, c->opts.grid_dims, nparts, levels, n, rp, ci)
          : partition_graph(nparts, levels, n, rp, ci);
  if (part.L > GS_MAX_LEVELS) throw Error(GS_EINVAL, "too many levels");
  if (c->opts.part_perm) c->nparts = (int)part.blocks[0].size() - 1;  // level-0 subdomains
  double t1 = now_s();
  extract_levels<T>(S->A, part, *S);
  check_rank<T>(*S, rank);
  T shift = T(0);
  if (c->opts.ilu_shift != 0.0) {
    if (!std::is_same<T, cplx>::value)
      throw Error(GS_EINVAL, "ilu_shift needs a complex matrix (the shifted factors are complex)");
    if (!std::isfinite(c->opts.ilu_shift)) throw Error(GS_EINVAL, "ilu_shift is not finite");
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t p = S->A.rp[i]; p < S->A.rp[i + 1]; ++p)
        if (S->A.ci[p] == i) sum += std::abs(S->A.v[p]);
    set_imag_shift(shift, c->opts.ilu_shift * sum / (double)n);
  }
  factor_levels<T>(*S, c->opts.ilu_kind, drop_tol, c->opts.lfil, c->opts.nthreads, shift);
  double t2 = now_s();
  if (std::is_same<T, double>::value) c->hd.reset((HostSetup<double>*)S.release());
  else c->hz.reset((HostSetup<cplx>*)S.release());
  c->eng = make_engine(host<T>(c), c->precision, c->stream);
  c->eng->set_inner(c->opts.inner_gmres_its);
  double t3 = now_s();
  HostSetup<T>& H = host<T>(c);
  if (!c->opts.defer_lowrank) {
    for (int l = H.L() - 1; l >= 0; --l) {
      if (l == H.L() - 1 && !c->opts.lowrank_last_level) continue;
      lowrank_level<T>(c, l, rank);
    }
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  double t4 = now_s();
  c->info = gs_info{};
  c->info.t_partition = t1 - t0;
  c->info.t_factor = t2 - t1;
  c->info.t_layout = t3 - t2;
  c->info.t_lowrank = t4 - t3;
  finish_setup<T>(c);
}

// a CSR block of an explicit level (rows x cols): rowptr present, from 0 and
// monotone, every column in range, col and val present when it has entries;
// checked before anything reads the block
static void check_block(const std::string& what, int64_t rows, int64_t cols, const int64_t* rp,
                        const int32_t* ci, const void* v) {
  if (!rp) throw Error(GS_EINVAL, what + ": NULL rowptr");
  if (rp[0] != 0) throw Error(GS_EINVAL, what + ": rowptr[0] != 0");
  for (int64_t i = 0; i < rows; ++i)
    if (rp[i + 1] < rp[i]) throw Error(GS_EINVAL, what + ": rowptr not monotone");
  const int64_t nnz = rp[rows];
  if (nnz > 0 && (!ci || !v)) throw Error(GS_EINVAL, what + ": NULL col or val");
  for (int64_t q = 0; q < nnz; ++q)
    if (ci[q] < 0 || ci[q] >= cols) throw Error(GS_EINVAL, what + ": column out of range");
}

template <class T>
static void setup_explicit(gs_ctx* c, int64_t n, const int64_t* rp, const int32_t* ci,
                           const void* val, const int64_t* perm, int nlevels,
                           const gs_level_data* L) {
  auto S = std::make_unique<HostSetup<T>>();
  copy_csr<T>(n, n, rp, ci, val, S->A);
  S->n = n;
  S->perm.assign(perm, perm + n);
  {
    std::vector<char> seen(n, 0);
    for (int64_t i = 0; i < n; ++i) {
      if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) throw Error(GS_EINVAL, "perm is not a permutation");
      seen[perm[i]] = 1;
    }
  }
  S->Ap = permute(S->A, S->perm);
  if (nlevels < 0 || nlevels > GS_MAX_LEVELS) throw Error(GS_EINVAL, "bad nlevels");
  int64_t start = 0;
  S->lv.resize(nlevels + 1);
  for (int l = 0; l <= nlevels; ++l) {
    const gs_level_data& a = L[l];
    HostLevel<T>& h = S->lv[l];
    h.start = start;
    h.d = a.d;
    h.s = n - start - a.d;
    if (a.d < 0 || h.s < 0) throw Error(GS_EINVAL, "level sizes exceed n");
    if (l == nlevels && h.s != 0) throw Error(GS_EINVAL, "level sizes do not add up to n");
    if (a.nblocks < 0 || !a.block_ptr) throw Error(GS_EINVAL, "missing block_ptr");
    h.blocks.assign(a.block_ptr, a.block_ptr + a.nblocks + 1);
    if (h.blocks.front() != 0 || h.blocks.back() != a.d) throw Error(GS_EINVAL, "block_ptr must span [0, d]");
    for (size_t b = 0; b + 1 < h.blocks.size(); ++b)
      if (h.blocks[b + 1] < h.blocks[b]) throw Error(GS_EINVAL, "block_ptr not monotone");
    const std::string tag = " of level " + std::to_string(l);
    check_block("L" + tag, a.d, a.d, a.l_rowptr, a.l_col, a.l_val);
    check_block("U" + tag, a.d, a.d, a.u_rowptr, a.u_col, a.u_val);
    if (a.d > 0) {
      validate_csr(a.d, a.u_rowptr, a.u_col, true);
      if (a.l_rowptr[a.d] > 0) validate_csr(a.d, a.l_rowptr, a.l_col, false);
    }
    copy_csr<T>(a.d, a.d, a.l_rowptr, a.l_col, a.l_val, h.L);
    copy_csr<T>(a.d, a.d, a.u_rowptr, a.u_col, a.u_val, h.U);
    if (h.s > 0) {
      check_block("E" + tag, h.s, a.d, a.e_rowptr, a.e_col, a.e_val);
      check_block("F" + tag, a.d, h.s, a.f_rowptr, a.f_col, a.f_val);
      copy_csr<T>(h.s, a.d, a.e_rowptr, a.e_col, a.e_val, h.E);
      copy_csr<T>(a.d, h.s, a.f_rowptr, a.f_col, a.f_val, h.F);
      h.k = a.k;
      // the low-rank kernels take k <= 1024, as check_rank does for gs_setup
      if (a.k < 0 || a.k > h.s || a.k > 1024)
        throw Error(GS_EINVAL, "bad rank on level " + std::to_string(l) + " (0 <= k <= min(s, 1024))");
      if (a.k > 0) {
        if (!a.w || !a.h) throw Error(GS_EINVAL, "NULL W or H" + tag);
        h.W.resize((size_t)h.s * a.k);
        h.H.resize((size_t)a.k * a.k);
        std::memcpy((void*)h.W.data(), a.w, h.W.size() * sizeof(T));
        std::memcpy((void*)h.H.data(), a.h, h.H.size() * sizeof(T));
      }
    } else {
      h.E.nrows = 0; h.E.ncols = a.d;
      h.F.nrows = a.d; h.F.ncols = 0;
      h.F.rp.assign(a.d + 1, 0);
    }
    start += a.d;
  }
  if (std::is_same<T, double>::value) c->hd.reset((HostSetup<double>*)S.release());
  else c->hz.reset((HostSetup<cplx>*)S.release());
  if (c->device >= 0) {
    c->eng = make_engine(host<T>(c), c->precision, c->stream);
    c->eng->set_inner(c->opts.inner_gmres_its);
  }
  c->info = gs_info{};
  finish_setup<T>(c);
}

// ------------------------------------------------------------ export / import
// File layout (little endian; "value" is 8 bytes for GS_F64, 16 for GS_C128
// as interleaved re, im; a CSR block is int64 nnz, int64 rowptr[rows + 1],
// int32 col[nnz], value val[nnz]):
//   char[8] "GEMSLR01", int32 dtype, int32 nlevels L, int64 n
//   CSR A (n rows, original numbering), int64 perm[n]
//   for l = 0 .. L: int64 d, int64 nblocks, int64 block_ptr[nblocks + 1],
//     CSR L_l (d rows), CSR U_l (d rows), and for l < L with
//     s = n - start_l - d: CSR E_l (s rows), CSR F_l (d rows), int32 k,
//     int32 0, value W_l[s k] (column-major), value H_l[k k] (column-major)
//   char[8] "GEMSLREN"
static const char kExportMagic[8] = {'G', 'E', 'M', 'S', 'L', 'R', '0', '1'};
static const char kExportEnd[8] = {'G', 'E', 'M', 'S', 'L', 'R', 'E', 'N'};

struct FileW {
  FILE* f;
  void put(const void* p, size_t n) {
    if (n && std::fwrite(p, 1, n, f) != n) throw Error(GS_EINVAL, "export: write failed");
  }
  template <class U> void put1(U v) { put(&v, sizeof(U)); }
};
struct FileR {
  FILE* f;
  void get(void* p, size_t n) {
    if (n && std::fread(p, 1, n, f) != n) throw Error(GS_EINVAL, "import: file truncated");
  }
  template <class U> U get1() {
    U v;
    get(&v, sizeof(U));
    return v;
  }
};

template <class T>
static void put_csr(FileW& w, const CSR<T>& m, int64_t rows) {
  if ((int64_t)m.rp.size() != rows + 1) throw Error(GS_EINVAL, "export: inconsistent CSR");
  w.put1<int64_t>(m.nnz());
  w.put(m.rp.data(), m.rp.size() * sizeof(int64_t));
  w.put(m.ci.data(), m.ci.size() * sizeof(int32_t));
  w.put((const void*)m.v.data(), m.v.size() * sizeof(T));
}

template <class T>
static void export_setup(const HostSetup<T>& S, int dtype, const char* path) {
  FILE* f = std::fopen(path, "wb");
  if (!f) throw Error(GS_EINVAL, std::string("export: cannot open ") + path);
  std::unique_ptr<FILE, int (*)(FILE*)> guard(f, std::fclose);
  FileW w{f};
  w.put(kExportMagic, 8);
  w.put1<int32_t>(dtype);
  w.put1<int32_t>(S.L());
  w.put1<int64_t>(S.n);
  put_csr(w, S.A, S.n);
  w.put(S.perm.data(), S.perm.size() * sizeof(int64_t));
  for (int l = 0; l <= S.L(); ++l) {
    const HostLevel<T>& h = S.lv[l];
    w.put1<int64_t>(h.d);
    w.put1<int64_t>((int64_t)h.blocks.size() - 1);
    w.put(h.blocks.data(), h.blocks.size() * sizeof(int64_t));
    put_csr(w, h.L, h.d);
    put_csr(w, h.U, h.d);
    if (l < S.L()) {
      put_csr(w, h.E, h.s);
      put_csr(w, h.F, h.d);
      w.put1<int32_t>(h.k);
      w.put1<int32_t>(0);
      w.put((const void*)h.W.data(), h.W.size() * sizeof(T));
      w.put((const void*)h.H.data(), h.H.size() * sizeof(T));
    }
  }
  w.put(kExportEnd, 8);
  // fclose flushes: report a failure there as well
  if (std::fclose(guard.release()) != 0) throw Error(GS_EINVAL, "export: write failed");
}

// Arrays of one CSR block read from a file (validated by setup_explicit).
template <class T>
struct CsrBuf {
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<T> v;
  void read(FileR& r, int64_t rows, int64_t limit) {
    const int64_t nnz = r.get1<int64_t>();
    if (rows < 0 || nnz < 0 || nnz > limit) throw Error(GS_EINVAL, "import: bad CSR size");
    rp.resize((size_t)rows + 1);
    r.get(rp.data(), rp.size() * sizeof(int64_t));
    if (rp[0] != 0 || rp[(size_t)rows] != nnz) throw Error(GS_EINVAL, "import: bad row pointers");
    for (int64_t i = 0; i < rows; ++i)
      if (rp[i + 1] < rp[i]) throw Error(GS_EINVAL, "import: bad row pointers");
    ci.resize((size_t)nnz);
    r.get(ci.data(), ci.size() * sizeof(int32_t));
    v.resize((size_t)nnz);
    r.get((void*)v.data(), v.size() * sizeof(T));
  }
};

template <class T>
static void import_setup(gs_ctx* c, const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) throw Error(GS_EINVAL, std::string("import: cannot open ") + path);
  std::unique_ptr<FILE, int (*)(FILE*)> guard(f, std::fclose);
  FileR r{f};
  char magic[8];
  r.get(magic, 8);
  if (std::memcmp(magic, kExportMagic, 8) != 0) throw Error(GS_EINVAL, "import: not a gs_export file");
  (void)r.get1<int32_t>();  // dtype, checked by the caller
  const int32_t L = r.get1<int32_t>();
  const int64_t n = r.get1<int64_t>();
  if (n <= 0 || L < 0 || L > GS_MAX_LEVELS) throw Error(GS_EINVAL, "import: bad header");
  // no array can hold more entries than the file has bytes
  std::fseek(f, 0, SEEK_END);
  const int64_t fsize = (int64_t)std::ftell(f);
  std::fseek(f, 24, SEEK_SET);
  if (n > fsize) throw Error(GS_EINVAL, "import: bad header");
  CsrBuf<T> A;
  A.read(r, n, fsize);
  std::vector<int64_t> perm((size_t)n);
  r.get(perm.data(), perm.size() * sizeof(int64_t));
  std::vector<std::vector<int64_t>> bp(L + 1);
  std::vector<CsrBuf<T>> Lf(L + 1), Uf(L + 1), Ef(L + 1), Ff(L + 1);
  std::vector<std::vector<T>> W(L + 1), H(L + 1);
  std::vector<gs_level_data> lv(L + 1);
  int64_t start = 0;
  for (int l = 0; l <= L; ++l) {
    gs_level_data& a = lv[l];
    std::memset(&a, 0, sizeof(a));
    a.d = r.get1<int64_t>();
    a.nblocks = r.get1<int64_t>();
    if (a.d < 0 || a.d > n - start || a.nblocks < 0 || a.nblocks > fsize)
      throw Error(GS_EINVAL, "import: bad level sizes");
    bp[l].resize((size_t)a.nblocks + 1);
    r.get(bp[l].data(), bp[l].size() * sizeof(int64_t));
    a.block_ptr = bp[l].data();
    Lf[l].read(r, a.d, fsize);
    Uf[l].read(r, a.d, fsize);
    a.l_rowptr = Lf[l].rp.data(); a.l_col = Lf[l].ci.data(); a.l_val = Lf[l].v.data();
    a.u_rowptr = Uf[l].rp.data(); a.u_col = Uf[l].ci.data(); a.u_val = Uf[l].v.data();
    const int64_t sl = n - start - a.d;
    if (l < L) {
      Ef[l].read(r, sl, fsize);
      Ff[l].read(r, a.d, fsize);
      a.e_rowptr = Ef[l].rp.data(); a.e_col = Ef[l].ci.data(); a.e_val = Ef[l].v.data();
      a.f_rowptr = Ff[l].rp.data(); a.f_col = Ff[l].ci.data(); a.f_val = Ff[l].v.data();
      a.k = r.get1<int32_t>();
      (void)r.get1<int32_t>();
      if (a.k < 0 || a.k > sl || (int64_t)a.k * sl > fsize) throw Error(GS_EINVAL, "import: bad rank");
      W[l].resize((size_t)sl * a.k);
      H[l].resize((size_t)a.k * a.k);
      r.get((void*)W[l].data(), W[l].size() * sizeof(T));
      r.get((void*)H[l].data(), H[l].size() * sizeof(T));
      a.w = W[l].data();
      a.h = H[l].data();
    }
    start += a.d;
  }
  char end[8];
  r.get(end, 8);
  if (std::memcmp(end, kExportEnd, 8) != 0) throw Error(GS_EINVAL, "import: bad end marker");
  guard.reset();
  validate_csr(n, A.rp.data(), A.ci.data(), false);
  setup_explicit<T>(c, n, A.rp.data(), A.ci.data(), A.v.data(), perm.data(), L, lv.data());
}


// ------------------------------------------------------------ learned start
template <class T>
static int features(gs_ctx* c, int l, float* X, int64_t rows_cap, int cols_cap) {
  HostSetup<T>& S = host<T>(c);
  if (l < 0 || l >= S.L()) throw Error(GS_EINVAL, "features: level out of range");
  const int nd = c->opts.grid_ndim;
  if (nd <= 0) throw Error(GS_EINVAL, "features need grid dimensions");
  const int NF = 38;
  const HostLevel<T>& h = S.lv[l];
  if (rows_cap < h.s || cols_cap < NF) throw Error(GS_EINVAL, "feature array too small");
  const int64_t n = S.n;
  int dims[3] = {1, 1, 1};
  for (int a = 0; a < nd; ++a) dims[a] = c->opts.grid_dims[a];
  int q = 1;
  while (true) {
    int64_t p = 1;
    for (int a = 0; a < nd; ++a) p *= (q + 1);
    if (p > c->nparts) break;
    ++q;
  }
  const CSR<T>& A = S.A;
  std::vector<double> ldiag(n, 0.0);
  double mean = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p)
      if (A.ci[p] == i) ldiag[i] = absval(A.v[p]);
    mean += ldiag[i];
  }
  mean /= (double)n;
  std::vector<double> lg(n);
  for (int64_t i = 0; i < n; ++i) lg[i] = std::log(std::max(ldiag[i], 1e-300) / mean);
  // E row sums and F column sums of level l (rows / columns indexed in C_l)
  std::vector<double> esum(h.s, 0.0), fsum(h.s, 0.0);
  for (int64_t j = 0; j < h.s; ++j)
    for (int64_t p = h.E.rp[j]; p < h.E.rp[j + 1]; ++p) esum[j] += absval(h.E.v[p]);
  for (int64_t i = 0; i < h.d; ++i)
    for (int64_t p = h.F.rp[i]; p < h.F.rp[i + 1]; ++p) fsum[h.F.ci[p]] += absval(h.F.v[p]);
  const int64_t stride[3] = {1, dims[0], (int64_t)dims[0] * dims[1]};
  const double pi = 3.14159265358979323846;
  for (int64_t j = 0; j < h.s; ++j) {
    const int64_t o = S.perm[h.start + h.d + j];
    float* f = X + (size_t)j * cols_cap;
    int crd[3] = {0, 0, 0};
    int64_t r = o;
    for (int a = 0; a < nd; ++a) { crd[a] = (int)(r % dims[a]); r /= dims[a]; }
    int fi = 0;
    double u[3];
    for (int a = 0; a < 3; ++a) {
      u[a] = a < nd ? (crd[a] + 1.0) / (dims[a] + 1.0) : 0.0;
      f[fi++] = (float)u[a];
    }
    for (int a = 0; a < 3; ++a)
      for (int m = 1; m <= 4; ++m) {
        f[fi++] = (float)std::sin(m * pi * u[a]);
        f[fi++] = (float)std::cos(m * pi * u[a]);
      }
    for (int a = 0; a < 3; ++a) {
      bool cut = false;
      if (a < nd)
        for (int jj = 1; jj < q; ++jj)
          if (crd[a] == (int)(((int64_t)jj * (dims[a] + 1)) / q)) cut = true;
      f[fi++] = cut ? 1.0f : 0.0f;
    }
    f[fi++] = (float)lg[o];
    double nsum = 0;
    int ncnt = 0;
    double conv[3] = {0, 0, 0};
    for (int64_t p = A.rp[o]; p < A.rp[o + 1]; ++p) {
      const int64_t cidx = A.ci[p];
      if (cidx == o) continue;
      nsum += lg[cidx];
      ++ncnt;
      for (int a = 0; a < nd; ++a) {
        if (cidx == o + stride[a]) conv[a] += realpart(A.v[p]);
        if (cidx == o - stride[a]) conv[a] -= realpart(A.v[p]);
      }
    }
    f[fi++] = (float)(ncnt ? nsum / ncnt : lg[o]);
    for (int a = 0; a < 3; ++a) f[fi++] = (float)(conv[a] / std::max(ldiag[o], 1e-300));
    f[fi++] = (float)(esum[j] / std::max(ldiag[o], 1e-300));
    f[fi++] = (float)(fsum[j] / std::max(ldiag[o], 1e-300));
    f[fi++] = (float)((double)l / (double)S.L());
    (void)fi;
  }
  return NF;
}

template <class T>
static void lowrank_all(gs_ctx* c, int rank, const float* const* warm) {
  HostSetup<T>& H = host<T>(c);
  check_rank<T>(H, rank);
  const double t0 = now_s();
  for (int l = H.L() - 1; l >= 0; --l) {
    HostLevel<T>& h = H.lv[l];
    h.k = 0;
    h.arnoldi_cycles = h.arnoldi_matvecs = h.arnoldi_converged = 0;
    c->eng->set_lowrank(l, 0, nullptr, nullptr);
    int method = 0;
    if (l == H.L() - 1 && !c->opts.lowrank_last_level) {
      c->info.lowrank_method[l] = 0;
      continue;
    }
    if (warm && warm[l] && c->opts.warm_start == 1) {
      method = 3;
      lowrank_level<T>(c, l, rank, warm[l]);
    } else if (warm && warm[l]) {
      method = 1;
      if (!lowrank_block<T>(c, l, rank, warm[l])) {
        const int used = h.arnoldi_matvecs;
        method = 2;
        lowrank_level<T>(c, l, rank);
        h.arnoldi_matvecs += used;
      }
    } else {
      lowrank_level<T>(c, l, rank);
    }
    if (l <= GS_MAX_LEVELS) c->info.lowrank_method[l] = method;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  c->info.t_lowrank = now_s() - t0;
  const double tl = c->info.t_lowrank;
  int methods[GS_MAX_LEVELS + 1];
  std::memcpy(methods, c->info.lowrank_method, sizeof(methods));
  const double tp = c->info.t_partition, tf = c->info.t_factor, ty = c->info.t_layout;
  finish_setup<T>(c);
  c->info.t_partition = tp;
  c->info.t_factor = tf;
  c->info.t_layout = ty;
  c->info.t_lowrank = tl;
  std::memcpy(c->info.lowrank_method, methods, sizeof(methods));
}

}  // namespace gs

// ====================================================================== C ABI
using namespace gs;

static void gs_set_err(gs_ctx* c, const char* m) {
  if (c) c->err = m;
  else g_create_error = m;
}

#define GS_GUARD(ctx, ...)                                   \
  try {                                                      \
    __VA_ARGS__;                                             \
  } catch (const Error& e) {                                 \
    gs_set_err((ctx), e.what());                             \
    return e.code;                                           \
  } catch (const std::bad_alloc&) {                          \
    gs_set_err((ctx), "host allocation failed");             \
    return GS_ENOMEM;                                        \
  } catch (const std::exception& e) {                        \
    gs_set_err((ctx), e.what());                             \
    return GS_EINVAL;                                        \
  }

template <class T>
static int ilu_host(int64_t n, const int64_t* rowptr, const int32_t* col, const void* val,
                    int kind, double tau, int lfil, int64_t* lrp, int32_t* lci, void* lv,
                    int64_t lcap, int64_t* urp, int32_t* uci, void* uv, int64_t ucap) {
  CSR<T> B, L, U;
  copy_csr<T>(n, n, rowptr, col, val, B);
  if (kind == GS_ILU0) ilu0(B, L, U);
  else if (kind == GS_ILUT) ilut(B, tau, lfil, L, U);
  else throw Error(GS_EINVAL, "unknown ILU kind");
  if (L.nnz() > lcap || U.nnz() > ucap) throw Error(GS_EINVAL, "output capacity too small");
  std::copy(L.rp.begin(), L.rp.end(), lrp);
  std::copy(U.rp.begin(), U.rp.end(), urp);
  std::copy(L.ci.begin(), L.ci.end(), lci);
  std::copy(U.ci.begin(), U.ci.end(), uci);
  std::memcpy(lv, (const void*)L.v.data(), L.v.size() * sizeof(T));
  std::memcpy(uv, (const void*)U.v.data(), U.v.size() * sizeof(T));
  return GS_OK;
}

template <class T>
static void level_sizes(const HostSetup<T>& S, int l, int64_t* z) {
  if (l < 0 || l > S.L()) throw Error(GS_EINVAL, "level out of range");
  const HostLevel<T>& h = S.lv[l];
  z[0] = h.d;
  z[1] = h.s;
  z[2] = (int64_t)h.blocks.size() - 1;
  z[3] = h.L.nnz();
  z[4] = h.U.nnz();
  z[5] = h.E.nnz();
  z[6] = h.F.nnz();
  z[7] = h.k;
}

template <class T>
static void level_copy(const HostSetup<T>& S, int l, int64_t* bp, int64_t* lrp, int32_t* lci,
                       void* lv, int64_t* urp, int32_t* uci, void* uv, int64_t* erp, int32_t* eci,
                       void* ev, int64_t* frp, int32_t* fci, void* fv, void* w, void* h) {
  if (l < 0 || l > S.L()) throw Error(GS_EINVAL, "level out of range");
  const HostLevel<T>& x = S.lv[l];
  auto cp = [](const CSR<T>& m, int64_t* rp, int32_t* ci, void* v) {
    if (rp) std::copy(m.rp.begin(), m.rp.end(), rp);
    if (ci) std::copy(m.ci.begin(), m.ci.end(), ci);
    if (v) std::memcpy(v, (const void*)m.v.data(), m.v.size() * sizeof(T));
  };
  if (bp) std::copy(x.blocks.begin(), x.blocks.end(), bp);
  cp(x.L, lrp, lci, lv);
  cp(x.U, urp, uci, uv);
  if (x.s > 0) {
    cp(x.E, erp, eci, ev);
    cp(x.F, frp, fci, fv);
  }
  if (w && !x.W.empty()) std::memcpy(w, (const void*)x.W.data(), x.W.size() * sizeof(T));
  if (h && !x.H.empty()) std::memcpy(h, (const void*)x.H.data(), x.H.size() * sizeof(T));
}

extern "C" {

void gs_opts_default(gs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->ilu_kind = GS_ILUT;
  o->lfil = 10;
  o->fgmres_restart = 50;
  o->maxit = 1000;
  o->arnoldi_tol = 1e-2;
  o->arnoldi_max_cycles = 20;
  o->lowrank_last_level = 1;
  o->precision = GS_PREC_F64;
  o->grid_ndim = 0;
  o->seed = 0;
  o->nthreads = 0;
  o->defer_lowrank = 0;
  o->block_max_iters = 8;
  o->inner_gmres_its = 0;
  o->ilu_shift = 0.0;
  o->warm_start = 0;
}

int gs_create(gs_ctx** ctx, int device, void* stream) {
  if (!ctx) return GS_EINVAL;
  *ctx = nullptr;
  auto c = std::make_unique<gs_ctx>();
  gs_opts_default(&c->opts);
  c->device = device;
  if (device >= 0) {
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
      g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
      return GS_EDEVICE;
    }
    c->stream = (hipStream_t)stream;
    e = resolve_scratch(device);
    if (e != hipSuccess) {
      g_create_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return GS_EDEVICE;
    }
  }
  *ctx = c.release();
  return GS_OK;
}

void gs_destroy(gs_ctx* c) {
  if (!c) return;
  if (c->device >= 0) {
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    c->eng.reset();
    c->amem.reset();
    c->wmem.reset();
    c->wkeep.clear();
    if (c->pin) (void)hipHostFree(c->pin);
    for (hipEvent_t e : c->fg_ev)
      if (e) (void)hipEventDestroy(e);
  }
  delete c;
}

const char* gs_last_error(const gs_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

static int need_device(gs_ctx* c) {
  if (!c) return GS_EINVAL;
  if (c->device < 0) {
    c->err = "host-only context";
    return GS_ESTATE;
  }
  hipcheck(hipSetDevice(c->device), "hipSetDevice");
  return GS_OK;
}

int gs_setup(gs_ctx* c, int64_t n, const int64_t* rowptr, const int32_t* col, const void* val,
             int dtype, int levels, int nparts, int rank, double drop_tol, const gs_opts* opts) {
  if (!c) return GS_EINVAL;
  // the partition arrays of opts are the caller's, read during this call
  // only: the kept options never point at them afterwards
  struct DropPartition {
    gs_opts& o;
    void clear() {
      o.part_perm = nullptr;
      o.part_level_start = nullptr;
      o.part_nlevels = 0;
      o.part_block_ptr = nullptr;
      o.part_block_count = nullptr;
    }
    ~DropPartition() { clear(); }
  } drop{c->opts};
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (opts) c->opts = *opts;
    else drop.clear();
    if (dtype != GS_F64 && dtype != GS_C128) throw Error(GS_EINVAL, "dtype must be GS_F64 or GS_C128");
    if (rank < 0 || ((levels < 1 || nparts < 1) && !c->opts.part_perm))
      throw Error(GS_EINVAL, "bad levels/nparts/rank");
    if (!val) throw Error(GS_EINVAL, "NULL values");
    validate_csr(n, rowptr, col, true);
    c->ready = false;
    c->eng.reset();
    c->hd.reset();
    c->hz.reset();
    c->dtype = dtype;
    c->precision = c->opts.precision;
    c->nparts = nparts;
    if (dtype == GS_F64) setup_native<double>(c, n, rowptr, col, val, levels, nparts, rank, drop_tol);
    else setup_native<cplx>(c, n, rowptr, col, val, levels, nparts, rank, drop_tol);
    return GS_OK;
  });
}

int gs_setup_explicit(gs_ctx* c, int64_t n, const int64_t* rowptr, const int32_t* col,
                      const void* val, int dtype, const int64_t* perm, int nlevels,
                      const gs_level_data* levels, const gs_opts* opts) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    // a host-only context keeps the host copy (export and inspection only)
    if (c->device >= 0) hipcheck(hipSetDevice(c->device), "hipSetDevice");
    if (opts) c->opts = *opts;
    if (dtype != GS_F64 && dtype != GS_C128) throw Error(GS_EINVAL, "dtype must be GS_F64 or GS_C128");
    if (!perm || !levels || !val) throw Error(GS_EINVAL, "NULL argument");
    validate_csr(n, rowptr, col, false);
    c->ready = false;
    c->eng.reset();
    c->hd.reset();
    c->hz.reset();
    c->dtype = dtype;
    c->precision = c->opts.precision;
    if (dtype == GS_F64) setup_explicit<double>(c, n, rowptr, col, val, perm, nlevels, levels);
    else setup_explicit<cplx>(c, n, rowptr, col, val, perm, nlevels, levels);
    return GS_OK;
  });
}

int gs_set_precision(gs_ctx* c, int precision) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (!c->ready) throw Error(GS_ESTATE, "no setup");
    if (precision == c->precision) return GS_OK;
    // the new engine is built from the host setup
    fetch_host_w_any(c);
    // build the new engine first: on error the current one stays in place
    std::unique_ptr<Engine> e = c->dtype == GS_F64 ? make_engine(*c->hd, precision, c->stream)
                                                   : make_engine(*c->hz, precision, c->stream);
    e->set_inner(c->opts.inner_gmres_its);
    c->eng = std::move(e);
    c->precision = precision;
    c->eng->stats(&c->info, 0);
    c->info.apply_bytes = c->eng->bytes_per_apply();
    return GS_OK;
  });
}

int gs_apply(gs_ctx* c, const void* x, void* y) { return gs_apply_many(c, 1, x, y); }

int gs_apply_many(gs_ctx* c, int nrhs, const void* x, void* y) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (!c->ready) throw Error(GS_ESTATE, "apply before setup");
    if (nrhs < 0) throw Error(GS_EINVAL, "negative nrhs");
    if (nrhs == 0) return GS_OK;  // an empty batch: nothing read or written
    if (!x || !y) throw Error(GS_EINVAL, "NULL vector");
    const int64_t n = c->dtype == GS_F64 ? c->hd->n : c->hz->n;
    const size_t vb = c->dtype == GS_F64 ? 8 : 16;
    const char* xb = (const char*)x;
    char* yb = (char*)y;
    const size_t bytes = (size_t)n * vb * (size_t)nrhs;
    if (xb < yb + bytes && yb < xb + bytes) throw Error(GS_EINVAL, "x and y alias");
    // several right-hand sides per factor pass (Sec. 6): every launch of a
    // level covers all vectors, and the triangular sweeps let groups of
    // vectors share each staged chunk of factor entries
    if (nrhs >= 2) c->eng->apply_batch(nrhs, xb, yb);
    else if (nrhs == 1) c->eng->apply(xb, yb, false);
    hipcheck(hipGetLastError(), "kernel launch");
    return GS_OK;
  });
}

int gs_apply_noalloc(gs_ctx* c, const void* x, void* y) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (!c->ready) throw Error(GS_ESTATE, "apply before setup");
    if (!x || !y) throw Error(GS_EINVAL, "NULL vector");
    const int64_t n = c->dtype == GS_F64 ? c->hd->n : c->hz->n;
    const size_t vb = c->dtype == GS_F64 ? 8 : 16;
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    const size_t bytes = (size_t)n * vb;
    if (xb < yb + bytes && yb < xb + bytes) throw Error(GS_EINVAL, "x and y alias");
    const size_t need = c->eng->scratch_bytes();
    if (need == 0)
      throw Error(GS_EINVAL, "gs_apply_noalloc: not available with inner GMRES steps");
    if (need > kStaticScratchBytes)
      throw Error(GS_EINVAL, "gs_apply_noalloc: this preconditioner needs " + std::to_string(need) +
                                 " bytes of scratch; the static region holds " +
                                 std::to_string(kStaticScratchBytes));
    void* base = c->device < kMaxDevices ? g_scratch_ptr[c->device] : nullptr;
    if (!base) throw Error(GS_EDEVICE, "static scratch not resolved for this device");
    c->eng->apply_in(x, y, base);
    hipcheck(hipGetLastError(), "kernel launch");
    return GS_OK;
  });
}

int gs_apply_profile(gs_ctx* c, const void* x, void* y, int reps, double* step_ms,
                     double* step_bytes, int cap, int* nsteps) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (!c->ready) throw Error(GS_ESTATE, "apply before setup");
    if (!x || !y || !step_ms || !step_bytes || !nsteps || reps < 1) throw Error(GS_EINVAL, "bad argument");
    std::vector<double> ms, by;
    std::vector<std::string> lab;
    const int ns = c->eng->profile(x, y, reps, ms, by, lab);
    if (ns > cap) throw Error(GS_EINVAL, "cap smaller than the number of launches");
    std::copy(ms.begin(), ms.end(), step_ms);
    std::copy(by.begin(), by.end(), step_bytes);
    c->step_labels = lab;
    *nsteps = ns;
    return GS_OK;
  });
}

const char* gs_apply_step_label(const gs_ctx* c, int i) {
  if (!c || i < 0 || i >= (int)c->step_labels.size()) return "";
  return c->step_labels[i].c_str();
}

int gs_probe_enable(gs_ctx* c, int kind, int max_launches) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (!c->ready) throw Error(GS_ESTATE, "no setup");
    if (max_launches < 0) throw Error(GS_EINVAL, "max_launches < 0");
    c->eng->probe_enable(kind, max_launches);
    return GS_OK;
  });
}

int gs_probe_read(gs_ctx* c, int64_t* launches, double* total_ms, double* total_bytes) {
  if (!c || !launches || !total_ms || !total_bytes) return GS_EINVAL;
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (!c->ready) throw Error(GS_ESTATE, "no setup");
    c->eng->probe_read(launches, total_ms, total_bytes);
    return GS_OK;
  });
}

int gs_solve(gs_ctx* c, const void* b, void* x, double tol, gs_info* info) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (!c->ready) throw Error(GS_ESTATE, "solve before setup");
    if (!b || !x) throw Error(GS_EINVAL, "NULL vector");
    if (!(tol > 0)) throw Error(GS_EINVAL, "tol must be positive");
    if (c->dtype == GS_F64) return fgmres<double>(c, b, x, tol, info);
    return fgmres<cplx>(c, b, x, tol, info);
  });
}


int gs_features(const gs_ctx* cc, int level, float* X, int64_t rows_cap, int cols_cap,
                int* ncols) {
  if (!cc || !X || !ncols) return GS_EINVAL;
  gs_ctx* c = const_cast<gs_ctx*>(cc);
  if (!c->ready) return GS_ESTATE;
  GS_GUARD(c, {
    *ncols = c->dtype == GS_F64 ? features<double>(c, level, X, rows_cap, cols_cap)
                                : features<cplx>(c, level, X, rows_cap, cols_cap);
    return GS_OK;
  });
}

int gs_lowrank(gs_ctx* c, int rank, const float* const* warm) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    int r = need_device(c);
    if (r) return r;
    if (!c->ready) throw Error(GS_ESTATE, "lowrank before setup");
    if (rank < 0) throw Error(GS_EINVAL, "rank < 0");
    if (c->dtype == GS_F64) lowrank_all<double>(c, rank, warm);
    else lowrank_all<cplx>(c, rank, warm);
    return GS_OK;
  });
}

int gs_get_info(const gs_ctx* c, gs_info* info) {
  if (!c || !info) return GS_EINVAL;
  if (!c->ready) return GS_ESTATE;
  *info = c->info;
  return GS_OK;
}

static int export_partition_impl(const Partition& p, int64_t* perm, int64_t* level_start,
                                 int* nlevels, int64_t* block_ptr, int64_t* block_count,
                                 int64_t block_cap);
static int export_partition(const Partition& p, int64_t* perm, int64_t* level_start,
                            int* nlevels, int64_t* block_ptr, int64_t* block_count,
                            int64_t block_cap) {
  return export_partition_impl(p, perm, level_start, nlevels, block_ptr, block_count, block_cap);
}

int gs_partition_grid(int ndim, const int32_t* dims, int nparts, int levels, int64_t n,
                      const int64_t* rowptr, const int32_t* col, int64_t* perm,
                      int64_t* level_start, int* nlevels, int64_t* block_ptr,
                      int64_t* block_count, int64_t block_cap) {
  gs_ctx* none = nullptr;
  GS_GUARD(none, {
    if (!perm || !level_start || !nlevels || !block_ptr || !block_count)
      throw Error(GS_EINVAL, "NULL output");
    validate_csr(n, rowptr, col, false);
    Partition p = partition_grid(ndim, dims, nparts, levels, n, rowptr, col);
    return export_partition(p, perm, level_start, nlevels, block_ptr, block_count, block_cap);
  });
}

int gs_partition_check(int64_t n, const int64_t* rowptr, const int32_t* col, const int64_t* perm,
                       const int64_t* level_start, int nlevels, const int64_t* block_ptr,
                       const int64_t* block_count, int64_t* block_ptr_out,
                       int64_t* block_count_out, int64_t block_cap) {
  gs_ctx* none = nullptr;
  GS_GUARD(none, {
    if (n <= 0) throw Error(GS_EINVAL, "n <= 0");
    validate_csr(n, rowptr, col, false);
    Partition p = user_partition(n, rowptr, col, perm, level_start, nlevels, block_ptr, block_count);
    if (!block_ptr_out || !block_count_out) return GS_OK;
    int64_t lvl[GS_MAX_LEVELS + 2];
    int64_t* pbuf = (int64_t*)std::malloc(sizeof(int64_t) * (size_t)n);
    if (!pbuf) throw std::bad_alloc();
    int nl = 0;
    const int rc = export_partition(p, pbuf, lvl, &nl, block_ptr_out, block_count_out, block_cap);
    std::free(pbuf);
    return rc;
  });
}

int gs_partition_graph(int nparts, int levels, int64_t n, const int64_t* rowptr,
                       const int32_t* col, int64_t* perm, int64_t* level_start, int* nlevels,
                       int64_t* block_ptr, int64_t* block_count, int64_t block_cap) {
  gs_ctx* none = nullptr;
  GS_GUARD(none, {
    if (!perm || !level_start || !nlevels || !block_ptr || !block_count)
      throw Error(GS_EINVAL, "NULL output");
    validate_csr(n, rowptr, col, false);
    Partition p = partition_graph(nparts, levels, n, rowptr, col);
    return export_partition(p, perm, level_start, nlevels, block_ptr, block_count, block_cap);
  });
}

static int export_partition_impl(const Partition& p, int64_t* perm, int64_t* level_start,
                                 int* nlevels, int64_t* block_ptr, int64_t* block_count,
                                 int64_t block_cap) {
  {
    int64_t need = 0;
    for (auto& b : p.blocks) need += (int64_t)b.size();
    if (need > block_cap) throw Error(GS_EINVAL, "block_cap too small");
    std::copy(p.perm.begin(), p.perm.end(), perm);
    std::copy(p.level_start.begin(), p.level_start.end(), level_start);
    *nlevels = p.L;
    int64_t pos = 0;
    for (size_t l = 0; l < p.blocks.size(); ++l) {
      block_count[l] = (int64_t)p.blocks[l].size() - 1;
      for (int64_t x : p.blocks[l]) block_ptr[pos++] = x;
    }
    return GS_OK;
  }
}

int gs_ilu(int64_t n, const int64_t* rowptr, const int32_t* col, const void* val, int dtype,
           int kind, double tau, int lfil, int64_t* l_rowptr, int32_t* l_col, void* l_val,
           int64_t l_cap, int64_t* u_rowptr, int32_t* u_col, void* u_val, int64_t u_cap) {
  gs_ctx* none = nullptr;
  GS_GUARD(none, {
    if (!val || !l_rowptr || !l_col || !l_val || !u_rowptr || !u_col || !u_val)
      throw Error(GS_EINVAL, "NULL argument");
    validate_csr(n, rowptr, col, false);
    if (dtype == GS_F64)
      return ilu_host<double>(n, rowptr, col, val, kind, tau, lfil, l_rowptr, l_col, l_val, l_cap,
                              u_rowptr, u_col, u_val, u_cap);
    if (dtype == GS_C128)
      return ilu_host<cplx>(n, rowptr, col, val, kind, tau, lfil, l_rowptr, l_col, l_val, l_cap,
                            u_rowptr, u_col, u_val, u_cap);
    throw Error(GS_EINVAL, "bad dtype");
  });
}

int gs_get_level_sizes(const gs_ctx* c, int l, int64_t* sizes) {
  if (!c || !sizes) return GS_EINVAL;
  if (!c->ready) return GS_ESTATE;
  gs_ctx* cc = const_cast<gs_ctx*>(c);
  GS_GUARD(cc, {
    if (c->dtype == GS_F64) level_sizes(*c->hd, l, sizes);
    else level_sizes(*c->hz, l, sizes);
    return GS_OK;
  });
}

int gs_get_level(const gs_ctx* c, int l, int64_t* block_ptr, int64_t* l_rowptr, int32_t* l_col,
                 void* l_val, int64_t* u_rowptr, int32_t* u_col, void* u_val, int64_t* e_rowptr,
                 int32_t* e_col, void* e_val, int64_t* f_rowptr, int32_t* f_col, void* f_val,
                 void* w, void* h) {
  if (!c) return GS_EINVAL;
  if (!c->ready) return GS_ESTATE;
  gs_ctx* cc = const_cast<gs_ctx*>(c);
  GS_GUARD(cc, {
    fetch_host_w_any(cc);  // a cache of the engine's W_l: the setup is unchanged
    if (c->dtype == GS_F64)
      level_copy(*c->hd, l, block_ptr, l_rowptr, l_col, l_val, u_rowptr, u_col, u_val, e_rowptr,
                 e_col, e_val, f_rowptr, f_col, f_val, w, h);
    else
      level_copy(*c->hz, l, block_ptr, l_rowptr, l_col, l_val, u_rowptr, u_col, u_val, e_rowptr,
                 e_col, e_val, f_rowptr, f_col, f_val, w, h);
    return GS_OK;
  });
}

int gs_get_perm(const gs_ctx* c, int64_t* perm) {
  if (!c || !perm) return GS_EINVAL;
  if (!c->ready) return GS_ESTATE;
  const std::vector<int64_t>& p = c->dtype == GS_F64 ? c->hd->perm : c->hz->perm;
  std::copy(p.begin(), p.end(), perm);
  return GS_OK;
}

int gs_export(const gs_ctx* c, const char* path) {
  if (!c) return GS_EINVAL;
  gs_ctx* cc = const_cast<gs_ctx*>(c);
  GS_GUARD(cc, {
    if (!c->ready) throw Error(GS_ESTATE, "export before setup");
    if (!path) throw Error(GS_EINVAL, "NULL path");
    fetch_host_w_any(cc);
    if (c->dtype == GS_F64) export_setup(*c->hd, GS_F64, path);
    else export_setup(*c->hz, GS_C128, path);
    return GS_OK;
  });
}

int gs_import(gs_ctx* c, const char* path, const gs_opts* opts) {
  if (!c) return GS_EINVAL;
  GS_GUARD(c, {
    if (!path) throw Error(GS_EINVAL, "NULL path");
    if (c->device >= 0) hipcheck(hipSetDevice(c->device), "hipSetDevice");
    int32_t dtype = -1;
    {
      FILE* f = std::fopen(path, "rb");
      if (!f) throw Error(GS_EINVAL, std::string("import: cannot open ") + path);
      char magic[8];
      const bool ok = std::fread(magic, 1, 8, f) == 8 && std::fread(&dtype, 4, 1, f) == 1;
      std::fclose(f);
      if (!ok || std::memcmp(magic, kExportMagic, 8) != 0)
        throw Error(GS_EINVAL, "import: not a gs_export file");
    }
    if (dtype != GS_F64 && dtype != GS_C128) throw Error(GS_EINVAL, "import: bad dtype");
    if (opts) c->opts = *opts;
    c->ready = false;
    c->eng.reset();
    c->hd.reset();
    c->hz.reset();
    c->dtype = dtype;
    c->precision = c->opts.precision;
    if (dtype == GS_F64) import_setup<double>(c, path);
    else import_setup<cplx>(c, path);
    return GS_OK;
  });
}

}  // extern "C"
