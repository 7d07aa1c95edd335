// Test driver for the host Schur routines of the low-rank setup: reads
// matrices from a binary file, writes their Schur factors.
//   input:  int32 count, then per matrix: int32 m, int32 is_complex,
//           m*m column-major values (double; complex: re, im pairs)
//   output: per matrix: m*m complex T, then m*m complex Q (re, im pairs)
// Real matrices go through schur_real, complex ones through schur_complex.
#include <cstdio>
#include <exception>
#include <vector>

#include "gs_internal.h"

static int run(int argc, char** argv);

int main(int argc, char** argv) {
  try {
    return run(argc, argv);
  } catch (const std::exception& e) {
    std::fprintf(stderr, "schur_driver: %s\n", e.what());
    return 5;
  }
}

static int run(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* in = std::fopen(argv[1], "rb");
  FILE* out = std::fopen(argv[2], "wb");
  if (!in || !out) return 3;
  int count = 0;
  if (std::fread(&count, 4, 1, in) != 1) return 4;
  for (int c = 0; c < count; ++c) {
    int hdr[2];
    if (std::fread(hdr, 4, 2, in) != 2) return 4;
    const int m = hdr[0];
    const size_t mm = (size_t)m * m;
    std::vector<gs::cplx> t, q;
    if (hdr[1]) {
      std::vector<double> raw(2 * mm);
      if (std::fread(raw.data(), 8, raw.size(), in) != raw.size()) return 4;
      t.resize(mm);
      for (size_t e = 0; e < mm; ++e) t[e] = gs::cplx(raw[2 * e], raw[2 * e + 1]);
      gs::schur_complex(m, t, q);
    } else {
      std::vector<double> a(mm);
      if (std::fread(a.data(), 8, a.size(), in) != a.size()) return 4;
      gs::schur_real(m, a, t, q);
    }
    std::fwrite(t.data(), sizeof(gs::cplx), mm, out);
    std::fwrite(q.data(), sizeof(gs::cplx), mm, out);
  }
  std::fclose(out);
  std::fclose(in);
  return 0;
}
