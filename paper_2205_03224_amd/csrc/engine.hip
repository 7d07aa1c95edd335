// Host orchestration of libgemslr: the level-scheduled device layout, the
// preconditioner apply (Alg. 2), the Ĝ_l matrix-vector product used by the
// low-rank setup (Sec. 4.2), thick-restart Arnoldi on the GPU, FGMRES, and
// the C ABI of include/gemslr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <functional>
#include <memory>
#include <string>
#include <thread>
#include <type_traits>

#include "device.h"
#include "engine.h"

namespace gs {

// ====================================================================== util

void hipcheck(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw Error(e == hipErrorOutOfMemory ? GS_ENOMEM : GS_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(x) hipcheck((x), #x)

DevMem::~DevMem() {
  for (void* p : ptrs) (void)hipFree(p);
}
void* DevMem::raw(size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) throw Error(GS_ENOMEM, "hipMalloc failed: " + std::string(hipGetErrorString(e)));
  ptrs.push_back(p);
  return p;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// storage conversions host value -> device storage
template <class V, class T> V to_store(const T& x);
template <> double to_store<double, double>(const double& x) { return x; }
template <> float to_store<float, double>(const double& x) { return (float)x; }
template <> bf16 to_store<bf16, double>(const double& x) {
  float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  bf16 b;
  b.u = (uint16_t)(u >> 16);
  return b;
}
template <> dcplx to_store<dcplx, cplx>(const cplx& x) { return mk(x.real(), x.imag()); }

template <class V, class T>
std::vector<V> convert(const std::vector<T>& h) {
  std::vector<V> out(h.size());
  for (size_t i = 0; i < h.size(); ++i) out[i] = to_store<V, T>(h[i]);
  return out;
}

// ====================================================================== layout

template <class T>
TriHost<T> build_tri(const CSR<T>& M, const std::vector<int64_t>& blocks, bool upper) {
  TriHost<T> h;
  std::vector<int> lev;
  std::vector<std::vector<int64_t>> bylev;
  std::vector<int64_t> rows;
  for (size_t b = 0; b + 1 < blocks.size(); ++b) {
    const int64_t r0 = blocks[b], r1 = blocks[b + 1], nr = r1 - r0;
    if (nr > 65535) throw Error(GS_EINVAL, "diagonal block larger than 65535 rows");
    lev.assign(nr, 0);
    int depth = 0;
    auto visit = [&](int64_t i) {
      int lv = 0;
      for (int64_t p = M.rp[i]; p < M.rp[i + 1]; ++p) {
        const int64_t c = M.ci[p];
        if (c < r0 || c >= r1) throw Error(GS_EINVAL, "factor entry outside its diagonal block");
        if (upper ? c > i : c < i) lv = std::max(lv, lev[c - r0] + 1);
      }
      lev[i - r0] = lv;
      depth = std::max(depth, lv + 1);
    };
    if (!upper) for (int64_t i = r0; i < r1; ++i) visit(i);
    else for (int64_t i = r1 - 1; i >= r0; --i) visit(i);
    h.depth = std::max(h.depth, depth);
    bylev.assign(depth, {});
    for (int64_t i = r0; i < r1; ++i) bylev[lev[i - r0]].push_back(i);
    for (const auto& rl : bylev) h.maxwidth = std::max(h.maxwidth, (int)rl.size());
    auto offd_count = [&](int64_t i) {
      int c = 0;
      for (int64_t p = M.rp[i]; p < M.rp[i + 1]; ++p)
        if (upper ? M.ci[p] > i : M.ci[p] < i) ++c;
      return c;
    };
    for (auto& rl : bylev) {
      std::stable_sort(rl.begin(), rl.end(), [&](int64_t x, int64_t y) {
        return offd_count(x) > offd_count(y);
      });
      for (size_t c0 = 0; c0 < rl.size(); c0 += 64) {
        const size_t c1 = std::min(rl.size(), c0 + 64);
        int maxnz = 0;
        std::vector<std::vector<std::pair<int32_t, T>>> ent(c1 - c0);
        for (size_t q = c0; q < c1; ++q) {
          const int64_t i = rl[q];
          T diag = T(0);
          bool hasdiag = false;
          for (int64_t p = M.rp[i]; p < M.rp[i + 1]; ++p) {
            const int64_t c = M.ci[p];
            if (c == i) { diag = M.v[p]; hasdiag = true; }
            else if (upper ? c > i : c < i) ent[q - c0].push_back({(int32_t)(c - r0), M.v[p]});
          }
          const int nz = (int)ent[q - c0].size();
          if (nz > 65535) throw Error(GS_EINVAL, "row too long");
          maxnz = std::max(maxnz, nz);
          h.rowinfo.push_back((uint32_t)(i - r0) | ((uint32_t)nz << 16));
          if (upper) {
            if (!hasdiag || absval(diag) == 0.0)
              throw Error(GS_EZEROPIVOT, "U factor has a zero or missing diagonal");
            h.dinv.push_back(T(1) / diag);
          }
        }
        h.maxslot = std::max(h.maxslot, maxnz);
        for (int j = 0; j < maxnz; ++j)
          for (size_t q = 0; q < ent.size(); ++q)
            if ((int)ent[q].size() > j) {
              h.val.push_back(ent[q][j].second);
              h.col.push_back((uint16_t)ent[q][j].first);
            }
        h.stage_row.push_back((int32_t)h.rowinfo.size());
        if (h.val.size() > (size_t)INT32_MAX) throw Error(GS_EINVAL, "factor too large");
        h.stage_ent.push_back((int32_t)h.val.size());
      }
    }
    h.blk_stage.push_back((int32_t)h.stage_row.size() - 1);
  }
  return h;
}


// Stages of the streamed sweep, by list scheduling per block: stage t takes
// up to `width` rows whose in-block dependencies all lie in earlier stages,
// longest remaining dependency chain first (ties: lower row), and passes
// over a row with more than `near_cap` entries in stage t - 1 (a stage
// later all of them are two back).  Every valid stage order gives the same
// solution; this one keeps the stage count near the dependency depth while
// bounding the stage width and the entries the sweep must gather after the
// previous stage's store.  Each row's entries are stored with those in
// stage t - 1 ("near") last, in column order otherwise; nnear records how
// many.  A stage for which every ready row is passed over holds one dummy
// row (index = block rows, no entries: the slot idle lanes store to).
template <class T>
TriHost<T> build_tri_sched(const CSR<T>& M, const std::vector<int64_t>& blocks, bool upper,
                           int width, int near_cap) {
  TriHost<T> h;
  std::vector<int32_t> dp, dc, sp, sc, height, rem, stage_of, cnt;
  std::vector<T> dval, diag;
  for (size_t b = 0; b + 1 < blocks.size(); ++b) {
    const int64_t r0 = blocks[b], r1 = blocks[b + 1];
    const int nr = (int)(r1 - r0);
    if (r1 - r0 > 65535) throw Error(GS_EINVAL, "diagonal block larger than 65535 rows");
    // in-block dependencies (off-diagonal entries of the triangle) and
    // their reverse
    dp.assign(nr + 1, 0);
    dc.clear();
    dval.clear();
    diag.assign(nr, T(0));
    std::vector<char> hasdiag(nr, 0);
    for (int i = 0; i < nr; ++i) {
      const int64_t gi = r0 + i;
      for (int64_t p = M.rp[gi]; p < M.rp[gi + 1]; ++p) {
        const int64_t c = M.ci[p];
        if (c < r0 || c >= r1) throw Error(GS_EINVAL, "factor entry outside its diagonal block");
        if (c == gi) {
          diag[i] = M.v[p];
          hasdiag[i] = 1;
        } else if (upper ? c > gi : c < gi) {
          dc.push_back((int32_t)(c - r0));
          dval.push_back(M.v[p]);
        }
      }
      dp[i + 1] = (int32_t)dc.size();
      if (dp[i + 1] - dp[i] > 65535) throw Error(GS_EINVAL, "row too long");
      h.maxslot = std::max(h.maxslot, dp[i + 1] - dp[i]);
    }
    sp.assign(nr + 1, 0);
    for (int32_t c : dc) ++sp[c + 1];
    for (int i = 0; i < nr; ++i) sp[i + 1] += sp[i];
    sc.assign(dc.size(), 0);
    {
      std::vector<int32_t> fill(sp.begin(), sp.end() - 1);
      for (int i = 0; i < nr; ++i)
        for (int32_t p = dp[i]; p < dp[i + 1]; ++p) sc[fill[dc[p]]++] = i;
    }
    // longest chain of dependents below each row (dependents come after it
    // in the sweep order: higher rows for L, lower for U)
    height.assign(nr, 1);
    int depth = 0;
    for (int k = 0; k < nr; ++k) {
      const int i = upper ? k : nr - 1 - k;
      for (int32_t p = sp[i]; p < sp[i + 1]; ++p) height[i] = std::max(height[i], height[sc[p]] + 1);
      depth = std::max(depth, height[i]);
    }
    h.depth = std::max(h.depth, depth);
    rem.assign(nr, 0);
    for (int i = 0; i < nr; ++i) rem[i] = dp[i + 1] - dp[i];
    stage_of.assign(nr, -1);
    // ready rows, best first: longest chain, then lower row
    auto worse = [&](int x, int y) { return height[x] != height[y] ? height[x] < height[y] : x > y; };
    std::vector<int> ready;
    for (int i = 0; i < nr; ++i)
      if (rem[i] == 0) ready.push_back(i);
    std::make_heap(ready.begin(), ready.end(), worse);
    std::vector<int> take, skip, fresh;
    int done = 0;
    for (int t = 0; done < nr; ++t) {
      take.clear();
      skip.clear();
      while (!ready.empty() && (int)take.size() < width) {
        std::pop_heap(ready.begin(), ready.end(), worse);
        const int i = ready.back();
        ready.pop_back();
        int near = 0;
        for (int32_t p = dp[i]; p < dp[i + 1]; ++p) near += stage_of[dc[p]] == t - 1;
        if (near > near_cap) skip.push_back(i);
        else take.push_back(i);
      }
      for (int i : skip) {
        ready.push_back(i);
        std::push_heap(ready.begin(), ready.end(), worse);
      }
      if (take.empty()) {
        // every ready row waits a stage: a stage of one dummy row
        h.rowinfo.push_back((uint32_t)nr);
        h.nnear.push_back(0);
        if (upper) h.dinv.push_back(T(1));
        h.stage_row.push_back((int32_t)h.rowinfo.size());
        h.stage_ent.push_back((int32_t)h.val.size());
        h.maxwidth = std::max(h.maxwidth, 1);
        continue;
      }
      for (int i : take) stage_of[i] = t;
      done += (int)take.size();
      h.maxwidth = std::max(h.maxwidth, (int)take.size());
      // rows with more entries first (slot-major storage below)
      std::stable_sort(take.begin(), take.end(), [&](int x, int y) {
        return dp[x + 1] - dp[x] > dp[y + 1] - dp[y];
      });
      std::vector<std::vector<std::pair<int32_t, T>>> ent(take.size());
      int maxnz = 0;
      for (size_t q = 0; q < take.size(); ++q) {
        const int i = take[q];
        int nn = 0;
        for (int pass = 0; pass < 2; ++pass)
          for (int32_t p = dp[i]; p < dp[i + 1]; ++p) {
            const bool nearp = stage_of[dc[p]] == t - 1;
            if (nearp != (pass == 1)) continue;
            ent[q].push_back({dc[p], dval[p]});
            nn += nearp;
          }
        const int nz = (int)ent[q].size();
        maxnz = std::max(maxnz, nz);
        h.rowinfo.push_back((uint32_t)i | ((uint32_t)nz << 16));
        h.nnear.push_back((uint8_t)nn);
        if (upper) {
          if (!hasdiag[i] || absval(diag[i]) == 0.0)
            throw Error(GS_EZEROPIVOT, "U factor has a zero or missing diagonal");
          h.dinv.push_back(T(1) / diag[i]);
        }
      }
      for (int j = 0; j < maxnz; ++j)
        for (size_t q = 0; q < ent.size(); ++q)
          if ((int)ent[q].size() > j) {
            h.val.push_back(ent[q][j].second);
            h.col.push_back((uint16_t)ent[q][j].first);
          }
      if (h.val.size() > (size_t)INT32_MAX) throw Error(GS_EINVAL, "factor too large");
      h.stage_row.push_back((int32_t)h.rowinfo.size());
      h.stage_ent.push_back((int32_t)h.val.size());
      // rows whose last dependency was scheduled become ready next stage
      fresh.clear();
      for (int i : take)
        for (int32_t p = sp[i]; p < sp[i + 1]; ++p)
          if (--rem[sc[p]] == 0) fresh.push_back(sc[p]);
      for (int i : fresh) {
        ready.push_back(i);
        std::push_heap(ready.begin(), ready.end(), worse);
      }
    }
    h.blk_stage.push_back((int32_t)h.stage_row.size() - 1);
  }
  return h;
}

// Pack the stages of every block (L stages, then U stages) into chunks of
// whole stages of at most `cap` bytes (see ChunkDesc).  Returns false if a
// single stage does not fit.
// Entry j of a row with cnt entries, the last nn of them near, goes to
// value slot slot_of(...) of the row (see near_slots): near entries fill the
// last slots of each lane's share (the low half first), far entries the
// remaining slots in order.  -1 if the row does not fit.
static int slot_of(int j, int cnt, int nn, int ms, bool half) {
  const int nfar = cnt - nn;
  if (cnt > ms || nn < 0 || nfar < 0) return -1;
  if (!half) {
    if (nn > near_slots(ms, false)) return -1;
    return j < nfar ? j : ms - cnt + j;
  }
  const int sl = ms / 2, nnh = near_slots(ms, true);
  const int klo = std::min(nn, nnh), khi = nn - klo;
  if (khi > nnh) return -1;
  if (j >= nfar) {
    const int u = j - nfar;
    return u < klo ? sl - klo + u : 2 * sl - khi + (u - klo);
  }
  const int flo = sl - klo;
  return j < flo ? j : sl + (j - flo);
}

template <class V, class D, class T>
bool build_chunks(const TriHost<T>& lo, const TriHost<T>& up, int b0, int b1, int cap, int ms,
                  int col_scale, int max_rows, bool half_l, bool half_u, std::vector<uint8_t>& blob,
                  std::vector<ChunkDesc>& desc, std::vector<int32_t>& blk_chunk) {
  auto pad = [](size_t x) { return (x + 15) & ~(size_t)15; };
  if (lo.nnear.size() != lo.rowinfo.size() || up.nnear.size() != up.rowinfo.size()) return false;
  // block-vector byte offsets of the columns (rows 0 .. max_rows - 1) must
  // fit the 16-bit column field
  if (max_rows > 0 && (size_t)(max_rows - 1) * (size_t)col_scale > 65535) return false;
  blob.clear();
  desc.clear();
  blk_chunk.assign(1, 0);
  for (int b = b0; b < b1; ++b) {
    for (int tri = 0; tri < 2; ++tri) {
      const TriHost<T>& h = tri == 0 ? lo : up;
      const bool isU = tri == 1;
      const bool half = isU ? half_u : half_l;
      const int sb = h.blk_stage[b], se = h.blk_stage[b + 1];
      const int VS = stream_vstride(ms), CS = stream_cstride(ms);
      auto size_of = [&](int s0, int s1) {
        const size_t rows = h.stage_row[s1] - h.stage_row[s0];
        return pad(rows * VS * sizeof(V)) + (isU ? pad(rows * sizeof(D)) : 0) +
               pad((rows + 1) * 4) + pad((rows + 1) * CS * 2);
      };
      int s = sb;
      while (s < se) {
        int s2 = s;
        while (s2 < se && size_of(s, s2 + 1) <= (size_t)cap) ++s2;
        if (s2 == s) return false;
        const size_t rows = h.stage_row[s2] - h.stage_row[s];
        if (rows > 65535) return false;
        ChunkDesc cd{};
        const size_t base = blob.size();
        if (base > 0xffffffffull) throw Error(GS_EINVAL, "level too large for 32-bit offsets");
        cd.off = (uint32_t)base;
        const size_t o_val = 0;
        const size_t o_dinv = pad(rows * VS * sizeof(V));
        const size_t o_info = o_dinv + (isU ? pad(rows * sizeof(D)) : 0);
        const size_t o_col = o_info + pad((rows + 1) * 4);  // zero word after the last row
        const size_t total = o_col + pad((rows + 1) * CS * 2);
        // the device copies whole 1 KiB rows of the chunk buffer
        if (total > (size_t)cap || cap % 1024 != 0) return false;
        cd.n16 = (uint16_t)(total / 16);
        cd.nst = (uint16_t)((s2 - s) | (isU ? 0x8000 : 0));
        cd.nrows = (uint16_t)rows;
        cd.dinv16 = (uint16_t)(o_dinv / 16);
        cd.info16 = (uint16_t)(o_info / 16);
        cd.col16 = (uint16_t)(o_col / 16);
        blob.resize(base + total, 0);  // zero values / columns for the padding
        uint8_t* p = blob.data() + base;
        const int32_t rb = h.stage_row[s];
        for (int k = s; k < s2; ++k) {
          const int32_t r0 = h.stage_row[k], r1 = h.stage_row[k + 1];
          const uint32_t nrs = (uint32_t)(r1 - r0);
          // compact slot-major source: slot j holds the rows with more than
          // j entries, which lead the stage (rows sorted by count)
          int32_t src = h.stage_ent[k];
          for (int j = 0; j < ms; ++j) {
            for (int32_t q = r0; q < r1; ++q) {
              const uint32_t cnt = (h.rowinfo[q] >> 16) & 0xffffu;
              if ((uint32_t)j >= cnt) continue;
              if (cnt > (uint32_t)ms) return false;
              const size_t row = (size_t)(q - rb);
              const V v = to_store<V, T>(h.val[src]);
              const uint16_t cb = (uint16_t)((uint32_t)h.col[src] * (uint32_t)col_scale);
              const int js = slot_of(j, (int)cnt, (int)h.nnear[q], ms, half);
              if (js < 0) return false;
              std::memcpy(p + o_val + (row * VS + js) * sizeof(V), &v, sizeof(V));
              // half-row stages: slots ms/2.. start at the next 4-byte
              // boundary of the column row (two lanes per row)
              const int hs = ms / 2, jc = (half && js >= hs) ? js - hs + stream_half_coff(ms) : js;
              std::memcpy(p + o_col + (row * CS + jc) * 2, &cb, 2);
              ++src;
            }
          }
          if (src != h.stage_ent[k + 1]) return false;
          for (int32_t q = r0; q < r1; ++q) {
            // the row's LDS byte offset in the block vector (24 bits) and
            // the stage's row count
            const uint32_t off = (h.rowinfo[q] & 0xffffu) * (uint32_t)col_scale;
            if (off > 0xffffffu || nrs > 255) return false;
            const uint32_t w = off | (nrs << 24);
            std::memcpy(p + o_info + (size_t)(q - rb) * 4, &w, 4);
            if (isU) {
              const D dv = to_store<D, T>(h.dinv[q]);
              std::memcpy(p + o_dinv + (size_t)(q - rb) * sizeof(D), &dv, sizeof(D));
            }
          }
        }
        desc.push_back(cd);
        s = s2;
      }
    }
    blk_chunk.push_back((int32_t)desc.size());
  }
  return true;
}

// most entries besides the diagonal in one row of a triangle
template <class T>
static int max_offdiag(const CSR<T>& M, bool upper) {
  int m = 0;
  for (int64_t i = 0; i + 1 < (int64_t)M.rp.size(); ++i) {
    int c = 0;
    for (int64_t p = M.rp[i]; p < M.rp[i + 1]; ++p) c += upper ? M.ci[p] > i : M.ci[p] < i;
    m = std::max(m, c);
  }
  return m;
}

// Diagonal blocks of a level swept by one workgroup.  Consecutive blocks are
// grouped: their union is still block diagonal, so its wavefront levels are
// the blocks' levels merged and every row is computed exactly as before,
// while one wavefront sweeps several blocks side by side (one sweep per CU
// runs faster per stage than several contending for it, and small blocks
// leave most lanes idle).  Only levels of small blocks (at most 1024 rows
// on average) are grouped: large blocks already fill the lanes, and pairing
// them measured slower (longer merged stages, one producer per CU).
// ceil(nb / CUs) blocks per group, as long as the group's 16-bit column
// offsets ((rows - 1) * elem <= 65535) and row indices hold.
static std::vector<int64_t> group_blocks(const std::vector<int64_t>& blocks, int num_cus,
                                         size_t elem) {
  const int64_t nb = (int64_t)blocks.size() - 1;
  if (nb <= num_cus || num_cus <= 0) return blocks;
  if (blocks[nb] - blocks[0] > 1024 * nb) return blocks;
  const int64_t per = (nb + num_cus - 1) / num_cus;
  const int64_t maxrows = std::min<int64_t>(65535 / (int64_t)elem + 1, 65535);
  std::vector<int64_t> g{blocks[0]};
  int64_t cnt = 0;
  for (int64_t b = 0; b < nb; ++b) {
    if (cnt > 0 && (cnt == per || blocks[b + 1] - g.back() > maxrows)) {
      g.push_back(blocks[b]);
      cnt = 0;
    }
    ++cnt;
  }
  g.push_back(blocks[nb]);
  return g;
}

// ---- the same two builders over block ranges on host threads, merged in
// block order (the result is identical to one sequential pass)
static int layout_threads(size_t nb) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  return (int)std::max<size_t>(1, std::min<size_t>({(size_t)hw, (size_t)16, nb / 8 + 1}));
}

// fn(sub-block list) builds the layout of those blocks (build_tri or
// build_tri_sched)
template <class T, class Fn>
TriHost<T> build_tri_par(const std::vector<int64_t>& blocks, Fn fn) {
  const size_t nb = blocks.size() - 1;
  const int nt = layout_threads(nb);
  if (nt <= 1) return fn(blocks);
  std::vector<TriHost<T>> part(nt);
  std::vector<std::exception_ptr> err(nt);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      try {
        const size_t b0 = nb * t / nt, b1 = nb * (t + 1) / nt;
        std::vector<int64_t> sub(blocks.begin() + b0, blocks.begin() + b1 + 1);
        part[t] = fn(sub);
      } catch (...) {
        err[t] = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  TriHost<T> h = std::move(part[0]);
  for (int t = 1; t < nt; ++t) {
    const TriHost<T>& q = part[t];
    const int32_t so = (int32_t)h.stage_row.size() - 1;
    const int32_t ro = (int32_t)h.rowinfo.size(), eo = (int32_t)h.val.size();
    for (size_t i = 1; i < q.blk_stage.size(); ++i) h.blk_stage.push_back(q.blk_stage[i] + so);
    for (size_t i = 1; i < q.stage_row.size(); ++i) h.stage_row.push_back(q.stage_row[i] + ro);
    for (size_t i = 1; i < q.stage_ent.size(); ++i) h.stage_ent.push_back(q.stage_ent[i] + eo);
    h.rowinfo.insert(h.rowinfo.end(), q.rowinfo.begin(), q.rowinfo.end());
    h.dinv.insert(h.dinv.end(), q.dinv.begin(), q.dinv.end());
    h.val.insert(h.val.end(), q.val.begin(), q.val.end());
    h.col.insert(h.col.end(), q.col.begin(), q.col.end());
    h.nnear.insert(h.nnear.end(), q.nnear.begin(), q.nnear.end());
    h.maxslot = std::max(h.maxslot, q.maxslot);
    h.depth = std::max(h.depth, q.depth);
    h.maxwidth = std::max(h.maxwidth, q.maxwidth);
  }
  return h;
}

template <class V, class D, class T>
bool build_chunks_par(const TriHost<T>& lo, const TriHost<T>& up, int nb, int cap, int ms,
                      int col_scale, int max_rows, bool half_l, bool half_u, std::vector<uint8_t>& blob,
                      std::vector<ChunkDesc>& desc, std::vector<int32_t>& blk_chunk) {
  const int nt = layout_threads((size_t)nb);
  std::vector<std::vector<uint8_t>> pb(nt);
  std::vector<std::vector<ChunkDesc>> pd(nt);
  std::vector<std::vector<int32_t>> pc(nt);
  std::vector<char> ok(nt, 0);
  std::vector<std::exception_ptr> err(nt);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      try {
        const int b0 = (int)((int64_t)nb * t / nt), b1 = (int)((int64_t)nb * (t + 1) / nt);
        ok[t] = build_chunks<V, D, T>(lo, up, b0, b1, cap, ms, col_scale, max_rows, half_l, half_u,
                                      pb[t], pd[t], pc[t]);
      } catch (...) {
        err[t] = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  for (char o : ok)
    if (!o) return false;
  blob.clear();
  desc.clear();
  blk_chunk.assign(1, 0);
  for (int t = 0; t < nt; ++t) {
    const size_t base = blob.size();
    if (base + pb[t].size() > 0xffffffffull) throw Error(GS_EINVAL, "level too large for 32-bit offsets");
    const int32_t d0 = (int32_t)desc.size();
    blob.insert(blob.end(), pb[t].begin(), pb[t].end());
    for (ChunkDesc cd : pd[t]) {
      cd.off += (uint32_t)base;
      desc.push_back(cd);
    }
    for (size_t i = 1; i < pc[t].size(); ++i) blk_chunk.push_back(pc[t][i] + d0);
  }
  return true;
}

// ====================================================================== engine

template <class P, class T>
struct EngineT final : Engine {
  using V = typename P::V;
  using C = typename P::C;
  using X = typename P::X;
  using D = typename P::D;
  using O = typename P::O;

  struct Lev {
    int64_t start = 0, d = 0, s = 0;
    int nb = 0, maxslot = 0, max_block_rows = 0, k = 0;
    int32_t* blk_row = nullptr;
    TriDev<P> lo{}, up{};
    CsrDev<P> E{}, F{};
    V* W = nullptr;
    C* H = nullptr;
    C* partial = nullptr;
    C* tprime = nullptr;
    int kcap = 0;
    int64_t nnz_lu = 0, nnz_e = 0, nnz_f = 0, nstages = 0;
    // streamed layout (null when the level uses the register-prefetch kernel)
    const uint8_t* blob = nullptr;
    const ChunkDesc* chunk = nullptr;
    const int32_t* blk_chunk = nullptr;
    int chunk_cap = 0, x_bytes = 0;
    bool half_l = false, half_u = false;  // L / U chunks laid out and swept as half rows
    D* diag_dinv = nullptr;  // diagonal level (L = I, U diagonal): 1/u_ii in row order
    int64_t nchunks = 0;
    int depth_l = 0, depth_u = 0;
    // F_l records of the streamed up sweep (null: F_l y2 by k_fy)
    const int32_t* frow = nullptr;
    const int32_t* fcol = nullptr;
    const V* fval = nullptr;
    const int32_t* funit = nullptr;
    int fw = 0;
    int64_t nrec = 0;
    // E_l records of the streamed down sweep (null: the interface step
    // gathers z1)
    const int32_t* erec = nullptr;
    const int32_t* eunit = nullptr;
    int64_t nerec = 0;
  };

  hipStream_t st;
  DevMem mem;
  int64_t n = 0;
  // measurement hooks (see Engine::profile / probe_enable)
  bool profiling = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<std::string> prof_label;
  std::vector<double> prof_bytes;
  std::vector<int> prof_kind;
  size_t prof_i = 0;
  int probe_kind = -1;
  std::vector<hipEvent_t> probe_ev;
  int64_t probe_n = 0;
  double probe_bytes_sum = 0;
  int32_t* perm_d = nullptr;
  X* t = nullptr;
  C* xg = nullptr;
  C* fy = nullptr;  // F_l y2 of the streamed up sweep
  int64_t fy_len = 0;
  X* ez = nullptr;  // z1 filed under E_l's entries by a down sweep (one level at a time)
  int64_t ez_len = 0;
  int max_lds = 65536;
  std::vector<Lev> lv;
  // several vectors per launch (ghat_batch, apply_batch): while nv > 1 the
  // working vector t (n rows per vector), fy (fy_len rows per vector) and
  // every level's partial / tprime are batch buffers of nv columns
  int nv = 1;
  std::unique_ptr<DevMem> bmem;
  int bcap = 0;
  std::vector<int> bk;  // the rank each level's batch partial / tprime were sized for
  X* tb = nullptr;
  C* fyb = nullptr;
  X* ezb = nullptr;
  std::vector<C*> partb, tpb;

  template <class U> U* upload(const std::vector<U>& h) {
    U* d = mem.alloc<U>(h.size());
    if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(U), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return d;
  }

  TriDev<P> upload_tri(const TriHost<T>& h, bool upper) {
    TriDev<P> d;
    d.blk_stage = upload(h.blk_stage);
    d.stage_row = upload(h.stage_row);
    d.stage_ent = upload(h.stage_ent);
    d.rowinfo = upload(h.rowinfo);
    d.dinv = upper ? upload(convert<D, T>(h.dinv)) : nullptr;
    d.val = upload(convert<V, T>(h.val));
    d.col = upload(h.col);
    return d;
  }

  CsrDev<P> upload_csr(const CSR<T>& m) {
    CsrDev<P> d;
    std::vector<int32_t> rp(m.rp.begin(), m.rp.end());
    d.rp = upload(rp);
    d.ci = upload(m.ci);
    d.v = upload(convert<V, T>(m.v));
    return d;
  }

  int lds_budget = 65536;  // LDS per workgroup of the streamed trisolve, at most
  int num_cus = 256, lds_per_cu = 163840;
  bool fixed_budget = false;
  bool no_stream = std::getenv("GEMSLR_NO_STREAM") != nullptr;
  // GEMSLR_NO_GROUP: one workgroup per diagonal block (no grouping);
  // GEMSLR_GROUP_CUS=c: group as if the device had c CUs (tests use it to
  // form groups from a few blocks)
  bool no_group = std::getenv("GEMSLR_NO_GROUP") != nullptr;
  // GEMSLR_NO_HALF: stages swept one lane per row even where two lanes per
  // row would pay
  bool no_half = std::getenv("GEMSLR_NO_HALF") != nullptr;
  // GEMSLR_NO_FUSE_SMALL: small levels use the three-launch interface step
  bool no_fuse_small = std::getenv("GEMSLR_NO_FUSE_SMALL") != nullptr;
  // GEMSLR_NO_FUSE_PERM: the apply gathers and scatters all n rows in
  // kernels of their own instead of inside the level-0 sweeps
  bool no_fuse_perm = std::getenv("GEMSLR_NO_FUSE_PERM") != nullptr;
  // GEMSLR_NO_FUSE_FY: F_l y2 of the streamed up sweep in a launch of its own
  bool no_fuse_fy = std::getenv("GEMSLR_NO_FUSE_FY") != nullptr;
  // GEMSLR_NO_FUSE_E: the interface step gathers z1 for E_l z1 instead of
  // reading what the down sweep filed under E_l's entries
  bool no_fuse_e = std::getenv("GEMSLR_NO_FUSE_E") != nullptr;
  // GEMSLR_NO_SMALL_LDS: the small-level interface step reads W_l and H_l
  // from global memory instead of copies in LDS
  bool no_small_lds = std::getenv("GEMSLR_NO_SMALL_LDS") != nullptr;
  // F_l records (see TriArgs::frow) of the sweep units grp: the rows that
  // hold entries, padded to the longest such row; none if a row is longer
  // than 16 entries (the sweep's prologue would then loop too long)
  void build_f_records(Lev& L, const CSR<T>& F, const std::vector<int64_t>& grp) {
    int64_t nrec = 0;
    int fw = 0;
    for (int64_t i = 0; i < L.d; ++i) {
      const int64_t len = F.rp[i + 1] - F.rp[i];
      if (len > 0) ++nrec;
      fw = std::max<int>(fw, (int)std::min<int64_t>(len, 1 << 20));
    }
    if (fw > 16) return;
    std::vector<int32_t> frow((size_t)nrec), funit((size_t)L.nb + 1, 0);
    std::vector<int32_t> fcol((size_t)(nrec * fw), 0);
    std::vector<T> fval((size_t)(nrec * fw), T(0));
    int64_t q = 0;
    for (int b = 0; b < L.nb; ++b) {
      funit[(size_t)b] = (int32_t)q;
      for (int64_t i = grp[b]; i < grp[b + 1]; ++i) {
        if (F.rp[i + 1] == F.rp[i]) continue;
        frow[(size_t)q] = (int32_t)(i - grp[b]);
        for (int64_t p = F.rp[i]; p < F.rp[i + 1]; ++p) {
          const int64_t j = p - F.rp[i];
          fcol[(size_t)(j * nrec + q)] = F.ci[p];
          fval[(size_t)(j * nrec + q)] = F.v[p];
        }
        ++q;
      }
    }
    funit[(size_t)L.nb] = (int32_t)q;
    L.frow = upload(frow);
    L.fcol = upload(fcol);
    L.fval = upload(convert<V, T>(fval));
    L.funit = upload(funit);
    L.fw = fw;
    L.nrec = nrec;
  }
  // E_l records (see TriArgs::erec) of the sweep units grp: every entry of
  // E_l, filed under the unit that holds its column, in entry order; none
  // if one unit's records would not fit a chunk buffer (they are staged
  // in the free one while the last chunk is swept)
  void build_e_records(Lev& L, const CSR<T>& E, const std::vector<int64_t>& grp) {
    const int nb = L.nb;
    const auto unit_of = [&](int64_t j) {
      return (int)(std::upper_bound(grp.begin(), grp.end(), j) - grp.begin()) - 1;
    };
    std::vector<int64_t> cnt((size_t)nb, 0);
    for (int32_t j : E.ci) ++cnt[(size_t)unit_of(j)];
    std::vector<int32_t> eunit((size_t)nb + 1, 0);
    int64_t tot = 0;
    for (int b = 0; b < nb; ++b) {
      const int64_t even = (cnt[(size_t)b] + 1) & ~(int64_t)1;
      if (even * 8 > L.chunk_cap) return;
      eunit[(size_t)b] = (int32_t)tot;
      tot += even;
    }
    if (tot >= ((int64_t)1 << 30)) return;
    eunit[(size_t)nb] = (int32_t)tot;
    std::vector<int32_t> rec((size_t)(2 * tot), 0);
    for (size_t q = 0; q < rec.size(); q += 2) rec[q] = -1;  // padding
    std::vector<int64_t> fill((size_t)nb, 0);
    for (int64_t p = 0; p < (int64_t)E.ci.size(); ++p) {
      const int b = unit_of(E.ci[(size_t)p]);
      const int64_t q = eunit[(size_t)b] + fill[(size_t)b]++;
      rec[(size_t)(2 * q)] = (int32_t)p;
      rec[(size_t)(2 * q + 1)] = (int32_t)(E.ci[(size_t)p] - grp[(size_t)b]);
    }
    L.erec = upload(rec);
    L.eunit = upload(eunit);
    L.nerec = tot;
  }
  // the down sweep of level l files z1 under E_l's entries for the
  // interface step that follows it
  bool ez_down(int l) const {
    return lv[l].erec && streamed(l) && lv[l].nb > 0 && l + 1 < (int)lv.size();
  }
  struct FusePerm {
    bool on = false;
    const O* x = nullptr;
    O* y = nullptr;
    const int32_t* perm = nullptr;
  } fuse;
  int group_cus = 256;
  // chunk buffers per workgroup: one chunk in flight while one is swept (a
  // third buffer, two in flight, measured slower: chunks a third smaller,
  // more hand-offs)
  static constexpr int chunk_bufs = 2;

  EngineT(const HostSetup<T>& S, hipStream_t stream) : st(stream) {
    n = S.n;
    {
      int dev = 0, maxlds = 65536;
      HIPCHK(hipGetDevice(&dev));
      if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        maxlds = 65536;
      // up to the device's per-workgroup limit (one group per CU); levels
      // with more groups than CUs share a CU's LDS below
      lds_budget = maxlds;
      max_lds = maxlds;
      int cus = 256, cu_lds = 163840;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
      if (hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                dev) != hipSuccess || cu_lds <= 0)
        cu_lds = 2 * lds_budget;
      num_cus = std::max(1, cus);
      group_cus = num_cus;
      if (const char* e = std::getenv("GEMSLR_GROUP_CUS")) group_cus = std::max(1, std::atoi(e));
      lds_per_cu = std::max(cu_lds, lds_budget);
      if (const char* e = std::getenv("GEMSLR_LDS_BUDGET")) {
        lds_budget = std::atoi(e);
        fixed_budget = true;
      }
    }
    std::vector<int32_t> p32(S.perm.begin(), S.perm.end());
    perm_d = upload(p32);
    t = mem.alloc<X>(n);
    int64_t maxd = 1;
    lv.resize(S.lv.size());
    for (size_t l = 0; l < S.lv.size(); ++l) {
      const HostLevel<T>& h = S.lv[l];
      Lev& L = lv[l];
      L.start = h.start;
      L.d = h.d;
      L.s = h.s;
      // the triangular solves sweep groups of consecutive blocks
      const std::vector<int64_t> grp =
          no_group ? h.blocks : group_blocks(h.blocks, group_cus, sizeof(C));
      L.nb = (int)grp.size() - 1;
      std::vector<int32_t> br(grp.begin(), grp.end());
      for (int b = 0; b < L.nb; ++b)
        L.max_block_rows = std::max<int>(L.max_block_rows, (int)(grp[b + 1] - grp[b]));
      L.blk_row = upload(br);
      // longest row of either triangle (entries besides the diagonal)
      L.maxslot = std::max(max_offdiag(h.L, false), max_offdiag(h.U, true));
      if (L.maxslot == 0 && h.d > 0) {
        // a diagonal level: keep 1/u_ii in row order (computed as the sweep
        // layout computes it), so a caller may fuse its solve
        std::vector<D> dv((size_t)h.d);
        for (int64_t i = 0; i < h.d; ++i) {
          T diag = T(0);
          for (int64_t p = h.U.rp[i]; p < h.U.rp[i + 1]; ++p)
            if (h.U.ci[p] == i) diag = h.U.v[p];
          if (absval(diag) == 0.0) throw Error(GS_EZEROPIVOT, "U factor has a zero or missing diagonal");
          dv[(size_t)i] = to_store<D, T>(T(1) / diag);
        }
        L.diag_dinv = upload(dv);
      }
      {
        // streamed layout: block vector and two chunk buffers in LDS, sized so
        // that two workgroups share one CU
        // (one slot more than the largest block: idle lanes store there)
        const int xb = (int)(((L.max_block_rows + 1) * sizeof(C) + 15) & ~(size_t)15);
        // LDS per workgroup: small enough that all groups of the level are
        // resident at once (ceil(nb / CUs) workgroups per CU)
        int budget = lds_budget;
        if (!fixed_budget && L.nb > 0) {
          const int per_cu = (L.nb + num_cus - 1) / num_cus;
          budget = std::min(lds_budget, lds_per_cu / std::max(1, per_cu));
          // two per CU when that keeps the largest chunks, so that launches
          // covering several vectors can double up where one vector leaves
          // CUs idle
          const int half = lds_per_cu / 2;
          if (per_cu == 1 && ((half - xb - 1024) / chunk_bufs) >= kChunkCapMax - 1024)
            budget = std::min(budget, half);
        }
        const auto cap_of = [&](int bgt) {
          return std::min(kChunkCapMax, ((bgt - xb - 1024) / chunk_bufs) & ~1023);
        };
        int cap = cap_of(budget);
        const int ms = stream_slots(L.maxslot);
        if (!no_stream && L.nb > 0 && ms > 0 &&
            cap_of(std::max(budget, std::min(lds_budget, lds_per_cu))) >= 4096) {
          // per triangle: half-row stages (at most 32 rows, two lanes per
          // row, each with half of the row's slots) unless they take more
          // than 8% more stages than full-row ones (at most 64 rows)
          auto sched = [&](const CSR<T>& M, bool upper, bool& half) {
            const int nf = near_slots(ms, false), nh = 2 * near_slots(ms, true);
            TriHost<T> full = build_tri_par<T>(grp, [&](const std::vector<int64_t>& sub) {
              return build_tri_sched(M, sub, upper, 64, nf);
            });
            half = false;
            if (no_half) return full;
            TriHost<T> hr = build_tri_par<T>(grp, [&](const std::vector<int64_t>& sub) {
              return build_tri_sched(M, sub, upper, 32, nh);
            });
            if ((hr.stage_row.size() - 1) * 100 <= (full.stage_row.size() - 1) * 108) {
              half = true;
              return hr;
            }
            return full;
          };
          bool hl = false, hu = false;
          TriHost<T> sl = sched(h.L, false, hl);
          TriHost<T> su = sched(h.U, true, hu);
          // Fewer workgroups per CU when co-residency would leave chunks of
          // fewer than three average stages: a chunk's copy then outlasts
          // its sweep and the copy latency shows (measured at level 0 of
          // the 128^3 workloads: complex128, 7 KB chunks at two workgroups
          // per CU 310 us per sweep, 24 KB chunks at one 262 us with two
          // rounds of blocks; float64 holds 3.4 stages in 7 KB chunks and
          // keeps two per CU)
          if (!fixed_budget && L.nb > 0) {
            const int nst = (int)(sl.stage_row.size() + su.stage_row.size()) - 2;
            const double row_bytes = stream_vstride(ms) * (double)sizeof(V) +
                                     stream_cstride(ms) * 2.0 + 4.0 + sizeof(D);
            const double stage_bytes = 2.0 * (double)L.d * row_bytes / std::max(1, nst);
            int per_cu = std::max(1, lds_per_cu / std::max(1, budget));
            while (cap < 3.0 * stage_bytes && cap < kChunkCapMax - 1024 && per_cu > 1) {
              --per_cu;
              budget = std::min(lds_budget, lds_per_cu / per_cu);
              cap = cap_of(budget);
            }
          }
          std::vector<uint8_t> blob;
          std::vector<ChunkDesc> desc;
          std::vector<int32_t> bc;
          if (cap >= 4096 &&
              build_chunks_par<V, D, T>(sl, su, L.nb, cap, ms, ColScale<C>::value,
                                        L.max_block_rows, hl, hu, blob, desc, bc)) {
            L.half_l = hl;
            L.half_u = hu;
            L.blob = upload(blob);
            std::vector<uint8_t> draw(desc.size() * sizeof(ChunkDesc));
            if (!desc.empty()) std::memcpy(draw.data(), desc.data(), draw.size());
            L.chunk = (const ChunkDesc*)upload(draw);
            L.blk_chunk = upload(bc);
            L.chunk_cap = cap;
            L.x_bytes = xb;
            L.nchunks = (int64_t)desc.size();
            L.depth_l = sl.depth;
            L.depth_u = su.depth;
            L.nstages = (int64_t)(sl.stage_row.size() + su.stage_row.size()) - 2;
          }
        }
      }
      // the per-stage layout feeds the register-prefetch kernel, used when
      // the streamed layout is unavailable or switched off
      if (!L.blob) {
        TriHost<T> tl = build_tri_par<T>(grp, [&](const std::vector<int64_t>& sub) {
          return build_tri(h.L, sub, false);
        });
        TriHost<T> tu = build_tri_par<T>(grp, [&](const std::vector<int64_t>& sub) {
          return build_tri(h.U, sub, true);
        });
        L.lo = upload_tri(tl, false);
        L.up = upload_tri(tu, true);
        L.depth_l = tl.depth;
        L.depth_u = tu.depth;
        L.nstages = (int64_t)(tl.stage_row.size() + tu.stage_row.size()) - 2;
      }
      L.nnz_lu = h.L.nnz() + h.U.nnz();
      if (h.s > 0) {
        L.E = upload_csr(h.E);
        L.F = upload_csr(h.F);
        L.nnz_e = h.E.nnz();
        L.nnz_f = h.F.nnz();
        if (L.blob && !no_fuse_fy && L.nnz_f > 0) build_f_records(L, h.F, grp);
        if (L.blob && !no_fuse_e && L.nnz_e > 0 && L.nnz_e < ((int64_t)1 << 30))
          build_e_records(L, h.E, grp);
      } else {
        std::vector<int32_t> zr(h.d + 1, 0);
        L.F.rp = upload(zr);
      }
      maxd = std::max(maxd, h.d);
      if (h.k > 0) {
        if (h.w_on_device) throw Error(GS_ESTATE, "W_l not fetched to the host before a rebuild");
        set_lowrank_host((int)l, h.k, h.W.data(), h.H.data());
      }
    }
    xg = mem.alloc<C>(maxd);
    fy = mem.alloc<C>(maxd);
    fy_len = maxd;
    for (const Lev& L : lv)
      if (L.erec) ez_len = std::max(ez_len, L.nnz_e);
    ez = mem.alloc<X>((size_t)std::max<int64_t>(ez_len, 1));
    // C_0 (the interface block of P^T A P) for the inner iteration's S_hat_0
    if constexpr (kInnerCapable) {
      if (lv.size() >= 2 && lv[0].s > 0) {
        const int64_t d0 = lv[0].d, s0 = lv[0].s;
        std::vector<int32_t> rp(1, 0), ci;
        std::vector<X> va;
        for (int64_t i = d0; i < n; ++i) {
          for (int64_t p = S.Ap.rp[i]; p < S.Ap.rp[i + 1]; ++p)
            if (S.Ap.ci[p] >= d0) {
              ci.push_back((int32_t)(S.Ap.ci[p] - d0));
              va.push_back(to_store<X, T>(S.Ap.v[p]));
            }
          rp.push_back((int32_t)ci.size());
        }
        (void)s0;
        c0_rp = upload(rp);
        c0_ci = upload(ci);
        c0_v = upload(va);
        c0_nnz = (int64_t)ci.size();
      }
    }
  }

  // ---- inner GMRES on S_hat_0 = C_0 - E_0 U_0^{-1} L_0^{-1} F_0 at the root
  // level (Alg. 2, l = 0), right-preconditioned by the l > 0 branch
  static constexpr bool kInnerCapable =
      std::is_same<X, double>::value || std::is_same<X, dcplx>::value;
  int inner_m = 0;
  std::unique_ptr<DevMem> imem;
  int32_t* c0_rp = nullptr;
  int32_t* c0_ci = nullptr;
  X* c0_v = nullptr;
  int64_t c0_nnz = 0;
  X *iV = nullptr, *iZ = nullptr, *iz1 = nullptr, *iw = nullptr, *ih = nullptr, *ipart = nullptr,
    *ihd = nullptr, *ic = nullptr;
  double *isub = nullptr, *iwn = nullptr, *inpart = nullptr, *ibeta = nullptr;

  void set_inner(int m) override {
    if (m <= 0 || lv.size() < 2 || lv[0].s == 0) {
      inner_m = 0;
      return;
    }
    if constexpr (!kInnerCapable) {
      throw Error(GS_EINVAL, "inner GMRES runs in the float64 / complex128 forms only");
    } else {
      if (m > kInnerMax) throw Error(GS_EINVAL, "inner GMRES: at most 16 steps");
      const int64_t d = lv[0].d, s = lv[0].s;
      imem = std::make_unique<DevMem>();
      iV = imem->alloc<X>((size_t)s * (m + 1));
      iZ = imem->alloc<X>((size_t)s * m);
      iz1 = imem->alloc<X>(std::max<int64_t>(d, 1));
      iw = imem->alloc<X>(s);
      ih = imem->alloc<X>((size_t)(m + 1) * m);
      ipart = imem->alloc<X>((size_t)256 * (m + 1));
      ihd = imem->alloc<X>(m + 1);
      ic = imem->alloc<X>(m);
      isub = imem->alloc<double>(m + 1);
      iwn = imem->alloc<double>(m + 1);
      inpart = imem->alloc<double>(256);
      ibeta = imem->alloc<double>(1);
      inner_m = m;
    }
  }

  // Root level with inner iterations: z1, z2 as usual, then m Arnoldi steps
  // on S_hat_0 P from v_0 = z2 / ||z2|| with P v = M_1^{-1}(v + W_0 H_0 W_0^H v)
  // and Z_j = P v_j kept, the small least-squares problem on the device,
  // y2 = Z c, and y1 = z1 - U^{-1} L^{-1} F y2.  Runs on the stream with no
  // host synchronisation.
  void inner_root() {
    if constexpr (kInnerCapable) {
      Lev& L = lv[0];
      const int64_t d = L.d, s = L.s;
      const int m = inner_m;
      X* tc = t + d;
      const X zx = zero_x();
      if (L.nb > 0)
        step("trisolve_down L0", KIND_TRI0, tri_bytes(0, TRI_DOWN), [&] { trisolve(0, TRI_DOWN); });
      interface(0, 0);
      launch_copy<X>(t, iz1, d, st);
      launch_norm<X>(tc, s, inpart, ibeta, st);
      launch_scale_inv<X>(tc, ibeta, iV, s, st);
      for (int j = 0; j < m; ++j) {
        X* vj = iV + (size_t)j * s;
        X* zj = iZ + (size_t)j * s;
        // z_j = P v_j
        launch_copy<X>(vj, tc, s, st);
        launch_fill<X>(t, zx, d, st);
        interface(0, L.k);
        run_from(1);
        launch_copy<X>(tc, zj, s, st);
        // w = C_0 z_j - E_0 U^{-1} L^{-1} F_0 z_j
        launch_fill<X>(t, zx, d, st);
        up(0);
        launch_spmv<X>(c0_rp, c0_ci, c0_v, zj, iw, s, st);
        launch_fill<X>(tc, zx, s, st);
        interface(0, 0);
        launch_sub<X>(iw, tc, iw, s, st);
        // Arnoldi step: two Gram-Schmidt passes, column j of Hbar
        launch_norm<X>(iw, s, inpart, iwn + j + 1, st);
        X* hj = ih + (size_t)j * (m + 1);
        launch_fill<X>(hj, zx, j + 1, st);
        for (int pass = 0; pass < 2; ++pass) {
          launch_multidot<X>(iV, s, j + 1, iw, s, ipart, ihd, st);
          launch_gemv_sub<X>(iV, s, j + 1, ihd, iw, s, hj, st);
        }
        launch_norm<X>(iw, s, inpart, isub + j + 1, st);
        launch_scale_inv<X>(iw, isub + j + 1, iV + (size_t)(j + 1) * s, s, st);
      }
      launch_inner_lsq<X>(ih, isub, iwn, ibeta, m, ic, st);
      launch_fill<X>(tc, zx, s, st);
      launch_gemv_add<X>(iZ, s, m, ic, tc, s, st);
      launch_copy<X>(iz1, t, d, st);
      up(0);
    }
  }

  // Install W_l, H_l; buffers grow with k and are reused by later calls.
  void set_lowrank_host(int l, int k, const T* W, const T* H) {
    lowrank_alloc(l, k);
    Lev& L = lv[l];
    std::vector<V> wv((size_t)L.s * k);
    for (size_t i = 0; i < wv.size(); ++i) wv[i] = to_store<V, T>(W[i]);
    std::vector<C> hc((size_t)k * k);
    for (size_t i = 0; i < hc.size(); ++i) hc[i] = to_compute(H[i]);
    if (!wv.empty())
      HIPCHK(hipMemcpyAsync(L.W, wv.data(), wv.size() * sizeof(V), hipMemcpyHostToDevice, st));
    if (!hc.empty())
      HIPCHK(hipMemcpyAsync(L.H, hc.data(), hc.size() * sizeof(C), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    L.k = k;
  }
  static C to_compute(const T& x);

  // W_l in the value type's own layout: float64 and complex128 storage
  static constexpr bool kExactW = sizeof(V) == sizeof(T);
  void lowrank_alloc(int l, int k) {
    Lev& L = lv[l];
    if (k > 1024) throw Error(GS_EINVAL, "rank above 1024 per level is not supported");
    if (k > L.kcap) {
      const int nblk = interface_blocks<P>(L.s);
      L.partial = mem.alloc<C>((size_t)nblk * k);
      L.tprime = mem.alloc<C>(k);
      L.W = mem.alloc<V>((size_t)L.s * k);
      L.H = mem.alloc<C>((size_t)k * k);
      L.kcap = k;
    }
  }
  int set_lowrank_device(int l, int k, const void* W, const void* H) override {
    lowrank_alloc(l, k);
    Lev& L = lv[l];
    const T* h = (const T*)H;
    std::vector<C> hc((size_t)k * k);
    for (size_t i = 0; i < hc.size(); ++i) hc[i] = to_compute(h[i]);
    if (L.s > 0 && k > 0) {
      if constexpr (kExactW) {
        HIPCHK(hipMemcpyAsync(L.W, W, (size_t)L.s * k * sizeof(V), hipMemcpyDeviceToDevice, st));
      } else {
        // narrower storage of a float64 setup
        launch_store_from_double<V>((const double*)W, L.W, (int64_t)L.s * k, st);
      }
    }
    if (!hc.empty())
      HIPCHK(hipMemcpyAsync(L.H, hc.data(), hc.size() * sizeof(C), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    L.k = k;
    return kExactW ? 1 : 0;
  }
  bool get_lowrank_w(int l, void* W) override {
    if (!kExactW) return false;
    const Lev& L = lv[l];
    if (L.s > 0 && L.k > 0)
      HIPCHK(hipMemcpyAsync(W, L.W, (size_t)L.s * L.k * sizeof(V), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return true;
  }
  void set_lowrank(int l, int k, const void* W, const void* H) override {
    const T* w = (const T*)W;
    const T* h = (const T*)H;
    set_lowrank_host(l, k, w, h);
  }

  TriArgs<P> tri_args(int l) {
    Lev& L = lv[l];
    TriArgs<P> a;
    a.lo = L.lo;
    a.up = L.up;
    a.blk_row = L.blk_row;
    a.t = t + L.start;
    a.d = L.d;
    a.F = L.F;
    a.xg = reinterpret_cast<X*>(xg);
    a.fy = fy;
    a.nb = L.nb;
    a.blob = L.blob;
    a.chunk = L.chunk;
    a.blk_chunk = L.blk_chunk;
    a.chunk_cap = L.chunk_cap;
    a.x_bytes = L.x_bytes;
    a.half_u = L.half_u ? 1 : 0;
    a.half_l = L.half_l ? 1 : 0;
    a.nvec = nv;
    a.ldt = nv > 1 ? n : 0;
    a.ldfy = nv > 1 ? fy_len : 0;
    a.xin = nullptr;
    a.yout = nullptr;
    a.perm = nullptr;
    a.ncons = 1;
    if (streamed(l) && L.frow) {
      a.frow = L.frow;
      a.fcol = L.fcol;
      a.fval = L.fval;
      a.funit = L.funit;
      a.fw = L.fw;
      a.nrec = L.nrec;
    }
    return a;
  }
  // Vectors per workgroup of the streamed sweep of level l for m vectors, as
  // (consumers, vectors) launches covering all m: each takes the consumer
  // count that sweeps the most vectors per round of co-resident workgroups
  // (LDS decides how many share a CU; every workgroup of a level is taken
  // to need the same time), the fewest consumers on ties.  A group of c
  // consumers reads the factor entries once for c vectors but holds c block
  // vectors in LDS, so it pays where the level's workgroups already fill
  // every CU (level 0) and not where one vector leaves CUs idle.
  std::vector<std::pair<int, int>> cons_plan(int l, int m) const {
    const Lev& L = lv[l];
    std::vector<std::pair<int, int>> plan;
    const int cmax = stream_max_cons((int)sizeof(C), stream_slots(L.maxslot));
    for (int r = m; r > 0;) {
      int best = 1;
      double brate = -1.0;
      for (int c = 1; c <= std::min(r, cmax); ++c) {
        const size_t lds = stream_lds_bytes(L.x_bytes, L.chunk_cap, c);
        if (lds > (size_t)max_lds) break;
        // co-resident workgroups per CU: LDS, and at most 32 waves
        const int64_t per_cu = std::min<int64_t>((int64_t)lds_per_cu / (int64_t)lds, 32 / (c + 1));
        if (per_cu < 1) break;
        const int64_t q = r / c;
        const int64_t slots = (int64_t)num_cus * per_cu;
        const int64_t rounds = ((int64_t)L.nb * q + slots - 1) / slots;
        const double rate = (double)(q * c) / (double)rounds;
        if (rate > brate * (1.0 + 1e-9)) {
          brate = rate;
          best = c;
        }
      }
      // GEMSLR_CONSUMERS=c: groups of c vectors wherever they fit (tests use
      // it where one vector per workgroup would be chosen)
      if (const char* e = std::getenv("GEMSLR_CONSUMERS")) {
        best = std::max(1, std::min({std::atoi(e), r, cmax}));
        while (best > 1 && stream_lds_bytes(L.x_bytes, L.chunk_cap, best) > (size_t)max_lds) --best;
      }
      const int cnt = (r / best) * best;
      plan.emplace_back(best, cnt);
      r -= cnt;
    }
    return plan;
  }
  bool streamed(int l) const { return lv[l].blob && !no_stream; }
  void trisolve(int l, int mode, bool ez_out = false) {
    const Lev& L = lv[l];
    if (streamed(l)) {
      TriArgs<P> a = tri_args(l);
      if (mode == TRI_DOWN && ez_out && L.erec) {
        a.erec = L.erec;
        a.eunit = L.eunit;
        a.ez = ez;
        a.ldez = nv > 1 ? ez_len : 0;
      }
      if (l == 0 && fuse.on) {
        // the apply's gather (scatter) of B_0 rows happens in this sweep, and
        // the up sweep also scatters the C_0 rows
        a.perm = fuse.perm;
        if (mode == TRI_DOWN) a.xin = fuse.x;
        else {
          a.yout = fuse.y;
          a.ccopy = nv == 1 ? L.s : 0;  // (fuse is on only for single applies)
        }
      }
      if (nv == 1) {
        launch_trisolve_streamed<P>(a, mode, L.maxslot, L.max_block_rows, st);
        return;
      }
      int j0 = 0;
      for (const auto& pc : cons_plan(l, nv)) {
        TriArgs<P> b = a;
        b.t += (int64_t)j0 * a.ldt;
        b.fy += (int64_t)j0 * a.ldfy;
        if (b.ez) b.ez += (int64_t)j0 * a.ldez;
        b.nvec = pc.second;
        b.ncons = pc.first;
        launch_trisolve_streamed<P>(b, mode, L.maxslot, L.max_block_rows, st);
        j0 += pc.second;
      }
    } else {
      launch_trisolve<P>(tri_args(l), mode, L.maxslot, L.max_block_rows, st);
    }
  }

  // Timing events take no system-scope fence: with one, each record writes
  // the L2s of all XCDs back to memory (measured: 11 us per apply for the
  // four events around the two level-0 sweeps, 4 us without the fence), time
  // the bracketed launch and the apply around it would be charged for. The
  // host reads the events only after a stream synchronisation.
  static constexpr unsigned kTimingEventFlags = hipEventDisableSystemFence;
  hipEvent_t ev_at(size_t i) {
    while (prof_ev.size() <= i) {
      hipEvent_t e;
      HIPCHK(hipEventCreateWithFlags(&e, kTimingEventFlags));
      prof_ev.push_back(e);
    }
    return prof_ev[i];
  }
  // Run one kernel launch; under measurement, bracket it with HIP events on
  // the engine's stream.
  template <class F>
  void step(const std::string& label, int kind, double bytes, F&& fn) {
    if (profiling) {
      HIPCHK(hipEventRecord(ev_at(2 * prof_i), st));
      fn();
      HIPCHK(hipEventRecord(ev_at(2 * prof_i + 1), st));
      if (prof_label.size() <= prof_i) {
        prof_label.push_back(label);
        prof_bytes.push_back(bytes);
        prof_kind.push_back(kind);
      }
      ++prof_i;
    } else if (kind == probe_kind && 2 * probe_n + 1 < (int64_t)probe_ev.size()) {
      HIPCHK(hipEventRecord(probe_ev[2 * probe_n], st));
      fn();
      HIPCHK(hipEventRecord(probe_ev[2 * probe_n + 1], st));
      probe_bytes_sum += bytes;
      ++probe_n;
    } else {
      fn();
    }
  }

  // ---- compulsory HBM bytes of each launch (every stored array read once,
  // every vector entry read or written once per touch)
  // the apply reads and writes the B_0 rows of the caller's vectors inside
  // the level-0 sweeps
  bool fuse_ok() const {
    // (level 0 must have an up sweep: it writes the B_0 rows of the result;
    // a one-level preconditioner ends with its down sweep)
    return inner_m == 0 && !no_fuse_perm && lv.size() > 1 && lv[0].d > 0 && lv[0].start == 0 &&
           streamed(0);
  }
  double tri_bytes(int l, int mode, bool perm_fused = false, bool ez_out = false) const {
    const Lev& L = lv[l];
    const double vb = sizeof(V), xb = sizeof(X), db = sizeof(D);
    // with the apply's permutation fused into level 0, the right-hand side
    // (DOWN) or the result (UP) is a caller vector entry plus its index
    const double fused = perm_fused ? (double)L.d * (4.0 + sizeof(O) - xb) : 0.0;
    double b = (double)(L.nnz_lu - L.d) * (vb + 2)   // factor value + 16-bit column
               + 2.0 * L.d * 4 + L.d * db              // row info (L and U), 1/u_ii
               + 4.0 * L.nstages + 8.0 * (L.nb + 1)    // stage and block tables
               + 2.0 * L.d * xb;                       // right-hand side in, result out
    // F_l: entries, then row pointers, or with the records the row of each
    // record and the unit table
    const double frows = streamed(l) && L.frow ? (double)L.nrec * 4 + (double)(L.nb + 1) * 4
                                               : (double)(L.d + 1) * 4;
    if (mode == TRI_UP)
      b += (double)L.nnz_f * (vb + 4) + frows                // F_l
           + (double)L.nnz_f * xb + (double)L.d * xb;        // y2 gathers, z1 read
    // the level-0 up sweep of an apply also scatters the C_0 rows
    if (perm_fused && mode == TRI_UP) b += perm_bytes(L.s);
    // the down sweep filing z1 under E_l's entries: records read, values written
    if (mode == TRI_DOWN && ez_out) b += 8.0 * L.nerec + 4.0 * (L.nb + 1) + (double)L.nnz_e * xb;
    return b + fused;
  }
  double if_bytes(int l, int k, bool gather_fused = false, bool ez_in = false) const {
    const Lev& L = lv[l];
    const double vb = sizeof(V), xb = sizeof(X);
    // gather fused: b2 is a caller vector entry plus its index
    const double b2 = gather_fused ? 4.0 + sizeof(O) : xb;
    // z1 filed in entry order: no column indices read
    const double ecol = ez_in ? 0.0 : 4.0;
    return (double)L.nnz_e * (vb + ecol) + (double)(L.s + 1) * 4 + (double)L.nnz_e * xb +
           (double)L.s * (b2 + xb) + (double)L.s * k * vb;
  }
  double upd_bytes(int l, int k) const {
    const Lev& L = lv[l];
    return (double)L.s * k * sizeof(V) + 2.0 * L.s * sizeof(X);
  }
  double perm_bytes(int64_t m) const { return (double)m * (4 + sizeof(O) + sizeof(X)); }

  // level l's small-level interface step can also do the solve of level
  // l + 1: the last level, diagonal, exactly level l's C-part
  bool last_fusable(int l) const {
    const Lev& L = lv[l];
    return !no_fuse_small && L.s <= 4096 && l + 2 == (int)lv.size() && lv[l + 1].diag_dinv &&
           lv[l + 1].start == L.start + L.d && lv[l + 1].d == L.s && lv[l].k <= 64;
  }
  // Returns true when the solve of level l + 1 (diagonal, the last level)
  // was done in the same launch (fuse_last requested and possible).
  bool interface(int l, int k, X* tv = nullptr, bool fuse_last = false, bool ez_in = false) {
    Lev& L = lv[l];
    if (!tv) tv = t;
    IfArgs<P> a;
    if (ez_in) {
      a.ez = ez;
      a.ldez = nv > 1 ? ez_len : 0;
    }
    a.E = L.E;
    a.t = tv + L.start;
    a.d = L.d;
    a.s = L.s;
    a.k = k;
    a.W = L.W;
    a.H = L.H;
    a.partial = L.partial;
    a.tprime = L.tprime;
    a.stage_w = no_small_lds ? 0 : 1;
    a.max_lds = max_lds;
    a.nvec = nv;
    a.ldt = nv > 1 ? n : 0;
    a.ldpart = nv > 1 ? (int64_t)interface_blocks<P>(L.s) * std::max(L.k, 1) : 0;
    const bool gfused = l == 0 && fuse.on && tv == t;
    if (gfused) {
      // the apply's gather of the C_0 rows happens here
      a.xin = fuse.x;
      a.perm = fuse.perm;
    }
    if (L.s <= 4096 && k <= 64 && !no_fuse_small) {
      // small level: the three steps in one workgroup (and, when the next
      // level is the last and diagonal, its solve)
      const bool last = fuse_last && last_fusable(l);
      if (last) a.last_dinv = lv[l + 1].diag_dinv;
      step(std::string(last ? "interface+update+solve L" : "interface+update L") +
               std::to_string(l),
           KIND_INTERFACE,
           if_bytes(l, k, gfused, ez_in) + (k > 0 ? upd_bytes(l, k) : 0.0) +
               (last ? (double)L.s * sizeof(D) : 0.0),
           [&] { launch_interface_small<P>(a, st); });
      return last;
    }
    step("interface L" + std::to_string(l), KIND_INTERFACE, if_bytes(l, k, gfused, ez_in),
         [&] { launch_interface<P>(a, st); });
    if (k > 0)
      step("lowrank_update L" + std::to_string(l), KIND_LOWRANK, upd_bytes(l, k),
           [&] {
             launch_lowrank_update<P>(tv + L.start + L.d, L.s, k, L.W, L.tprime, st, nv,
                                      nv > 1 ? n : 0);
           });
    return false;
  }

  // returns true when the last level's solve was fused into this level's
  // interface step
  bool down(int l) {
    const bool ezl = ez_down(l);
    if (lv[l].nb > 0)
      step("trisolve_down L" + std::to_string(l), l == 0 ? KIND_TRI0 : KIND_TRI,
           tri_bytes(l, TRI_DOWN, l == 0 && fuse.on, ezl), [&] {
             trisolve(l, TRI_DOWN, ezl);
           });
    if (l + 1 < (int)lv.size()) return interface(l, lv[l].k, nullptr, !no_fuse_small, ezl);
    return false;
  }
  void up(int l) {
    if (lv[l].nb > 0)
      step("trisolve_up L" + std::to_string(l), l == 0 ? KIND_TRI0 : KIND_TRI,
           tri_bytes(l, TRI_UP, l == 0 && fuse.on), [&] {
             trisolve(l, TRI_UP);
           });
  }
  void run_from(int l0) {
    const int L = (int)lv.size() - 1;
    bool last_done = false;
    for (int l = l0; l <= L; ++l) {
      if (l == L && last_done) break;
      last_done = down(l);
    }
    for (int l = L - 1; l >= l0; --l) up(l);
  }

  void apply(const void* x, void* y, bool permuted) override {
    const int32_t* pm = permuted ? nullptr : perm_d;
    const int64_t d0 = lv.empty() ? 0 : lv[0].d;
    if (fuse_ok()) {
      // B_0 rows are read and written by the level-0 sweeps themselves, the
      // C_0 rows read by the level-0 interface step and written by the
      // level-0 up sweep
      const O* xo = (const O*)x;
      O* yo = (O*)y;
      fuse = {true, xo, yo, pm};
      run_from(0);
      fuse = {};
      return;
    }
    step("gather", KIND_PERM, perm_bytes(n),
         [&] { launch_gather<P>((const O*)x, pm, t, n, st); });
    if (inner_m > 0) inner_root();
    else run_from(0);
    step("scatter", KIND_PERM, perm_bytes(n),
         [&] { launch_scatter<P>(t, pm, (O*)y, n, st); });
  }

  // ---- the apply on a caller's scratch region (see Engine::apply_in)
  static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }
  // rows of the global block-vector staging (blocks too large for LDS in
  // the register-prefetch sweep) and of F_l y2 staging (up sweeps that take
  // F_l y2 from a launch of its own)
  int64_t xg_need() const {
    int64_t m = 0;
    for (const Lev& L : lv)
      if (L.nb > 0 && !streamed((int)(&L - lv.data())) &&
          (size_t)L.max_block_rows * sizeof(C) > 65536)
        m = std::max(m, L.d);
    return m;
  }
  int64_t fy_need() const {
    int64_t m = 0;
    for (size_t l = 0; l + 1 < lv.size(); ++l)
      if (lv[l].nb > 0 && streamed((int)l) && !lv[l].frow) m = std::max(m, lv[l].d);
    return m;
  }
  size_t scratch_bytes() const override {
    if (inner_m > 0) return 0;
    size_t b = up256((size_t)n * sizeof(X)) + up256((size_t)xg_need() * sizeof(C)) +
               up256((size_t)fy_need() * sizeof(C)) + up256((size_t)ez_len * sizeof(X));
    for (const Lev& L : lv)
      if (L.k > 0)
        b += up256((size_t)interface_blocks<P>(L.s) * L.k * sizeof(C)) + up256((size_t)L.k * sizeof(C));
    return std::max<size_t>(b, 256);
  }
  void apply_in(const void* x, void* y, void* base) override {
    if (inner_m > 0) throw Error(GS_EINVAL, "inner GMRES steps keep their own work space");
    uint8_t* p = (uint8_t*)base;
    auto take = [&](size_t bytes) {
      void* q = p;
      p += up256(bytes);
      return q;
    };
    X* const t0 = t;
    C* const xg0 = xg;
    C* const fy0 = fy;
    X* const ez0 = ez;
    C* part0[GS_MAX_LEVELS + 2];
    C* tp0[GS_MAX_LEVELS + 2];
    const size_t nl = std::min(lv.size(), (size_t)GS_MAX_LEVELS + 2);
    t = (X*)take((size_t)n * sizeof(X));
    xg = (C*)take((size_t)xg_need() * sizeof(C));
    fy = (C*)take((size_t)fy_need() * sizeof(C));
    ez = (X*)take((size_t)ez_len * sizeof(X));
    for (size_t l = 0; l < nl; ++l) {
      Lev& L = lv[l];
      part0[l] = L.partial;
      tp0[l] = L.tprime;
      if (L.k > 0) {
        L.partial = (C*)take((size_t)interface_blocks<P>(L.s) * L.k * sizeof(C));
        L.tprime = (C*)take((size_t)L.k * sizeof(C));
      }
    }
    auto restore = [&] {
      t = t0;
      xg = xg0;
      fy = fy0;
      ez = ez0;
      for (size_t l = 0; l < nl; ++l) {
        lv[l].partial = part0[l];
        lv[l].tprime = tp0[l];
      }
    };
    try {
      apply(x, y, false);
    } catch (...) {
      restore();
      throw;
    }
    restore();
  }

  int profile(const void* x, void* y, int reps, std::vector<double>& ms,
              std::vector<double>& bytes, std::vector<std::string>& labels) override {
    profiling = true;
    std::vector<double> acc;
    for (int r = 0; r < reps; ++r) {
      prof_i = 0;
      apply(x, y, false);
      HIPCHK(hipStreamSynchronize(st));
      acc.resize(prof_i, 0.0);
      for (size_t i = 0; i < prof_i; ++i) {
        float e = 0;
        HIPCHK(hipEventElapsedTime(&e, prof_ev[2 * i], prof_ev[2 * i + 1]));
        acc[i] += e;
      }
    }
    profiling = false;
    ms.assign(acc.size(), 0.0);
    for (size_t i = 0; i < acc.size(); ++i) ms[i] = acc[i] / std::max(1, reps);
    bytes.assign(prof_bytes.begin(), prof_bytes.begin() + acc.size());
    labels.assign(prof_label.begin(), prof_label.begin() + acc.size());
    return (int)acc.size();
  }

  void probe_enable(int kind, int max_launches) override {
    for (hipEvent_t e : probe_ev) (void)hipEventDestroy(e);
    probe_ev.clear();
    probe_kind = kind;
    probe_n = 0;
    probe_bytes_sum = 0;
    for (int i = 0; i < 2 * std::max(0, max_launches) + 1 && kind >= 0; ++i) {
      hipEvent_t e;
      HIPCHK(hipEventCreateWithFlags(&e, kTimingEventFlags));
      probe_ev.push_back(e);
    }
  }
  void probe_read(int64_t* launches, double* ms, double* bytes) override {
    HIPCHK(hipStreamSynchronize(st));
    double tot = 0;
    for (int64_t i = 0; i < probe_n; ++i) {
      float e = 0;
      HIPCHK(hipEventElapsedTime(&e, probe_ev[2 * i], probe_ev[2 * i + 1]));
      tot += e;
    }
    *launches = probe_n;
    *ms = tot;
    *bytes = probe_bytes_sum;
    probe_n = 0;
    probe_bytes_sum = 0;
  }

  ~EngineT() override {
    (void)hipStreamSynchronize(st);
    for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : probe_ev) (void)hipEventDestroy(e);
  }

  void ghat(int l, const void* v, void* out) override {
    Lev& L = lv[l];
    X* tc = t + L.start + L.d;
    launch_gather<P>((const O*)v, nullptr, tc, L.s, st);
    run_from(l + 1);
    launch_fill<X>(t + L.start, zero_x(), L.d, st);
    up(l);
    launch_fill<X>(tc, zero_x(), L.s, st);
    interface(l, 0);
    launch_scatter<P>(tc, nullptr, (O*)out, L.s, st);
  }

  // ---- several vectors per launch
  static constexpr int kBatchMax = 64;
  void batch_reserve(int m) {
    // a level's rank can grow after the buffers were made (a low-rank term
    // installed after a batched product, as the block iteration does level
    // by level): then they are made again, for the ranks now in place
    bool fits = m <= bcap && bk.size() == lv.size();
    for (size_t l = 0; fits && l < lv.size(); ++l) fits = lv[l].k <= bk[l];
    if (fits) return;
    m = std::max(m, bcap);
    bmem.reset();
    bmem = std::make_unique<DevMem>();
    tb = bmem->alloc<X>((size_t)n * m);
    fyb = bmem->alloc<C>((size_t)std::max<int64_t>(fy_len, 1) * m);
    ezb = bmem->alloc<X>((size_t)std::max<int64_t>(ez_len, 1) * m);
    partb.assign(lv.size(), nullptr);
    tpb.assign(lv.size(), nullptr);
    bk.assign(lv.size(), 0);
    for (size_t l = 0; l < lv.size(); ++l)
      if (lv[l].k > 0) {
        partb[l] = bmem->alloc<C>((size_t)interface_blocks<P>(lv[l].s) * lv[l].k * m);
        tpb[l] = bmem->alloc<C>((size_t)lv[l].k * m);
        bk[l] = lv[l].k;
      }
    bcap = m;
  }
  // run f with the batch buffers of m vectors in place of t, fy, partial,
  // tprime (restored afterwards, also on error)
  template <class Fn>
  void with_batch(int m, Fn f) {
    batch_reserve(m);
    X* const t0 = t;
    C* const fy0 = fy;
    X* const ez0 = ez;
    std::vector<C*> p0(lv.size()), q0(lv.size());
    for (size_t l = 0; l < lv.size(); ++l) {
      p0[l] = lv[l].partial;
      q0[l] = lv[l].tprime;
      if (lv[l].k > 0) {
        lv[l].partial = partb[l];
        lv[l].tprime = tpb[l];
      }
    }
    t = tb;
    fy = fyb;
    ez = ezb;
    nv = m;
    auto restore = [&] {
      t = t0;
      fy = fy0;
      ez = ez0;
      nv = 1;
      for (size_t l = 0; l < lv.size(); ++l) {
        lv[l].partial = p0[l];
        lv[l].tprime = q0[l];
      }
    };
    try {
      f();
    } catch (...) {
      restore();
      throw;
    }
    restore();
  }
  // out[:, j] = G_hat_l v[:, j] for m vectors of s_l entries each (column
  // j at v + j * s_l), every launch of a level covering all m vectors;
  // each column equals ghat of that column
  void ghat_batch(int l, int m, const void* v, void* out) override {
    if (m <= 0) return;
    if (inner_m > 0 || m == 1) {
      const size_t vb = sizeof(O) * (size_t)lv[l].s;
      for (int j = 0; j < m; ++j) ghat(l, (const char*)v + j * vb, (char*)out + j * vb);
      return;
    }
    for (int j0 = 0; j0 < m; j0 += kBatchMax) {
      const int mm = std::min(kBatchMax, m - j0);
      with_batch(mm, [&] {
        Lev& L = lv[l];
        const O* vv = (const O*)v + (size_t)j0 * L.s;
        O* oo = (O*)out + (size_t)j0 * L.s;
        for (int j = 0; j < mm; ++j)
          launch_gather<P>(vv + (size_t)j * L.s, nullptr, t + (size_t)j * n + L.start + L.d, L.s,
                           st);
        run_from(l + 1);
        for (int j = 0; j < mm; ++j) launch_fill<X>(t + (size_t)j * n + L.start, zero_x(), L.d, st);
        up(l);
        for (int j = 0; j < mm; ++j)
          launch_fill<X>(t + (size_t)j * n + L.start + L.d, zero_x(), L.s, st);
        interface(l, 0);
        for (int j = 0; j < mm; ++j)
          launch_scatter<P>(t + (size_t)j * n + L.start + L.d, nullptr, oo + (size_t)j * L.s, L.s,
                            st);
      });
    }
  }
  // y[:, j] = M^{-1} x[:, j] for m vectors of n entries (original order),
  // every launch of a level covering all m vectors; each column equals
  // apply of that column
  void apply_batch(int m, const void* x, void* y) override {
    if (m <= 0) return;
    if (inner_m > 0) {
      for (int j = 0; j < m; ++j)
        apply((const O*)x + (size_t)j * n, (O*)y + (size_t)j * n, false);
      return;
    }
    for (int j0 = 0; j0 < m; j0 += kBatchMax) {
      const int mm = std::min(kBatchMax, m - j0);
      with_batch(mm, [&] {
        const O* xx = (const O*)x + (size_t)j0 * n;
        O* yy = (O*)y + (size_t)j0 * n;
        for (int j = 0; j < mm; ++j)
          launch_gather<P>(xx + (size_t)j * n, perm_d, t + (size_t)j * n, n, st);
        run_from(0);
        for (int j = 0; j < mm; ++j)
          launch_scatter<P>(t + (size_t)j * n, perm_d, yy + (size_t)j * n, n, st);
      });
    }
  }
  static X zero_x();

  void stats(gs_info* info, int vb_vec) override {
    (void)vb_vec;
    for (size_t l = 0; l < lv.size() && l <= GS_MAX_LEVELS; ++l) {
      info->depth_l[l] = lv[l].depth_l;
      info->depth_u[l] = lv[l].depth_u;
    }
  }

  // Compulsory HBM traffic of one whole apply: the sum over its launches.
  double bytes_per_apply() const override {
    if (fuse_ok()) return apply_bytes_from(0, true);
    double b = 2 * perm_bytes(n);
    if (inner_m > 0) {
      // root level with inner steps: down + interface, per step one product
      // with P (interface with W, levels >= 1) and one with S_hat_0 (up,
      // interface, C_0) plus the Arnoldi vectors, then the final up
      const Lev& R = lv[0];
      const double xb = sizeof(X);
      const double lower = apply_bytes_from(1);
      double step_b = if_bytes(0, R.k) + upd_bytes(0, R.k) + lower + tri_bytes(0, TRI_UP) +
                      if_bytes(0, 0) + (double)c0_nnz * (xb + 4) + (double)(R.s + 1) * 4;
      b += tri_bytes(0, TRI_DOWN) + if_bytes(0, 0) + tri_bytes(0, TRI_UP);
      for (int j = 0; j < inner_m; ++j) b += step_b + (double)R.s * xb * (2.0 * (j + 1) * 2 + 8);
      b += (double)R.s * xb * (inner_m + 2);
      return b;
    }
    return b + apply_bytes_from(0);
  }
  // bytes of run_from(l0)
  double apply_bytes_from(int l0, bool perm_fused = false) const {
    double b = 0;
    const int L = (int)lv.size() - 1;
    for (int l = l0; l <= L; ++l) {
      const bool f = perm_fused && l == 0;
      if (l == L && l > l0 && last_fusable(l - 1)) {
        b += (double)lv[l].d * sizeof(D);  // 1/u_ii read by the fused solve
        break;
      }
      const bool e = ez_down(l);
      if (lv[l].nb > 0) b += tri_bytes(l, TRI_DOWN, f, e);
      if (l < L) {
        b += if_bytes(l, lv[l].k, f, e);
        if (lv[l].k > 0) b += upd_bytes(l, lv[l].k);
        if (lv[l].nb > 0) b += tri_bytes(l, TRI_UP, f);
      }
    }
    return b;
  }
};

template <> double EngineT<PF64, double>::to_compute(const double& x) { return x; }
template <> float EngineT<PF32, double>::to_compute(const double& x) { return (float)x; }
template <> float EngineT<PBF16, double>::to_compute(const double& x) { return (float)x; }
template <> dcplx EngineT<PC128, cplx>::to_compute(const cplx& x) { return mk(x.real(), x.imag()); }
template <> double EngineT<PF64, double>::zero_x() { return 0.0; }
template <> float EngineT<PF32, double>::zero_x() { return 0.0f; }
template <> float EngineT<PBF16, double>::zero_x() { return 0.0f; }
template <> dcplx EngineT<PC128, cplx>::zero_x() { return mk(0, 0); }

std::unique_ptr<Engine> make_engine(const HostSetup<double>& S, int precision, hipStream_t st) {
  if (precision == GS_PREC_F64) return std::make_unique<EngineT<PF64, double>>(S, st);
  if (precision == GS_PREC_F32) return std::make_unique<EngineT<PF32, double>>(S, st);
  if (precision == GS_PREC_BF16) return std::make_unique<EngineT<PBF16, double>>(S, st);
  throw Error(GS_EINVAL, "unknown precision");
}
std::unique_ptr<Engine> make_engine(const HostSetup<cplx>& S, int precision, hipStream_t st) {
  if (precision != GS_PREC_F64) throw Error(GS_EINVAL, "complex data supports GS_PREC_F64 only");
  return std::make_unique<EngineT<PC128, cplx>>(S, st);
}

}  // namespace gs
