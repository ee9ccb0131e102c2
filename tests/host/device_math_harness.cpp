// Host build of the device math of the coefficient path (the same headers the
// kernels include), driven from tests/test_host_device_code.py.
//   sincos <x...>            : prints sin, cos of each x with sincos_bounded
//   sincosm <x...>           : the same with sincos_moderate
//   roots  (stdin problem)   : prints u, b, status of find_root for each pair, then
//                              the root record's e^{-b}, 1 - e^{-b} and the sine
//                              and cosine of half the offset from the 2M grid
//   tunecache <path>         : writes two autotuner cache entries to path, reads
//                              them back and prints them; then reads path as it
//                              is after a test has altered it
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ffbie_root.hpp"
#include "ffbie_tuning_cache.hpp"

using namespace ffbie;

static double table_sin(int i, int M) {
  const int n = 8 * M;
  i %= n;
  if (i < 0) i += n;
  int sign = 1;
  if (i >= 4 * M) { i -= 4 * M; sign = -1; }
  if (i > 2 * M) i = 4 * M - i;
  long double v = (i <= M) ? sinl((long double)M_PI * i / (4.0L * M))
                           : cosl((long double)M_PI * (2 * M - i) / (4.0L * M));
  return sign * (double)v;
}

static void print_entries(const std::vector<TuneEntry>& v) {
  printf("%zu\n", v.size());
  for (const TuneEntry& e : v)
    printf("%s|%d|%s|%d|%d|%d|%d|%.6g\n", e.device.c_str(), e.M, e.precision.c_str(), e.t.fft_radix,
           e.t.pairs_per_item, e.t.waves_per_block, e.t.persistent, e.main_ms);
}

int main(int argc, char** argv) {
  if (argc > 2 && !strcmp(argv[1], "tunecache")) {
    if (argc > 3 && !strcmp(argv[3], "read")) {
      print_entries(tune_cache_read(argv[2]));
      return 0;
    }
    std::vector<TuneEntry> v(2);
    v[0].device = "gfx950 x256"; v[0].M = 64; v[0].precision = "f64";
    v[0].t = ffbie_tuning{2, 16, 4, 0}; v[0].main_ms = 12.5;
    v[1].device = "gfx950 x256"; v[1].M = 128; v[1].precision = "f32";
    v[1].t = ffbie_tuning{4, 8, 2, 1}; v[1].main_ms = 0.25;
    if (!tune_cache_write(argv[2], v)) return 2;
    const std::vector<TuneEntry> r = tune_cache_read(argv[2]);
    print_entries(r);
    const TuneEntry* h = tune_cache_find(r, "gfx950 x256", 128, "f32");
    const TuneEntry* miss = tune_cache_find(r, "gfx950 x256", 128, "f64");
    printf("%d %d\n", h ? h->t.fft_radix : -1, miss ? 1 : 0);
    return 0;
  }
  if (argc > 1 && (!strcmp(argv[1], "sincos") || !strcmp(argv[1], "sincosm"))) {
    const bool moderate = !strcmp(argv[1], "sincosm");
    double x;
    while (scanf("%lf", &x) == 1) {
      double s, c;
      if (moderate) sincos_moderate(x, &s, &c);
      else sincos_bounded(x, &s, &c);
      printf("%.17g %.17g\n", s, c);
    }
    return 0;
  }
  int M, lmax, mmax;
  double k;
  if (scanf("%d %lf %d %d", &M, &k, &lmax, &mmax) != 4) return 1;
  Prob P{};
  P.M = M; P.M0 = M; P.L = 2 * M; P.tab_n = 8 * M; P.k = k; P.eps0 = 1e-15;
  P.g.lmax = lmax; P.g.mmax = mmax;
  P.g.ax[0] = P.g.ax[1] = P.g.ax[2] = 1.0;
  for (int l = 0; l < lmax; ++l)
    for (int m = 0; m <= mmax; ++m)
      if (scanf("%lf", &P.g.a[l][m]) != 1) return 1;
  std::vector<double> tab(P.tab_n);
  for (int i = 0; i < P.tab_n; ++i) tab[i] = table_sin(i, M);
  int n;
  if (scanf("%d", &n) != 1) return 1;
  for (int i = 0; i < n; ++i) {
    double t, ts;
    int j;
    if (scanf("%lf %d %lf", &t, &j, &ts) != 3) return 1;
    int st = 0;
    RootRec r;
    if (mmax <= 0) r = find_root<0>(P, tab.data(), t, j, ts, &st);
    else if (mmax <= 2) r = find_root<2>(P, tab.data(), t, j, ts, &st);
    else if (mmax <= 4) r = find_root<4>(P, tab.data(), t, j, ts, &st);
    else r = find_root<8>(P, tab.data(), t, j, ts, &st);
    printf("%.17g %.17g %d %.17g %.17g %.17g %.17g\n", r.u, r.b, st, r.eb, r.omq, r.sh, r.ch);
  }
  return 0;
}
