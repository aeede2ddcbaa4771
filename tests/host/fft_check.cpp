// The line transforms of csrc/pgx_fft.hpp run on the CPU: every lane of a
// line is a std::thread, the synchronisation between the LDS exchanges a
// std::barrier, the LDS line a host array with guard entries.  For every
// shape the kernels use (two- and three-stage Stockham schedules),
// both directions, FP32 and FP64, and both twiddle sources, the result is
// compared with a direct DFT in long double.  Built with ThreadSanitizer, the
// run also shows that no two lanes touch one line entry between two
// barriers; with AddressSanitizer, that no lane leaves its line.  Exits
// non-zero on the first failed check.
#include <barrier>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_1705_03464_amd/csrc/pgx_fft.hpp"

using namespace pgx;

#define CHECK(c, ...)                                              \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s: ", #c);              \
      std::fprintf(stderr, __VA_ARGS__);                           \
      std::fprintf(stderr, "\n");                                  \
      std::exit(1);                                                \
    }                                                              \
  } while (0)

// per-stage twiddles exp(-2 pi i r k / (Ns R)) at [twoff(s) + r Ns + k],
// computed in FP64 and rounded to T (as the library's host code does)
template <typename Sh, typename T> std::vector<C<T>> twiddles() {
  std::vector<C<T>> h(Sh::tw_entries());
  for (int st = 1; st < Sh::stages; ++st) {
    const int R = Sh::radix(st), Ns = Sh::ns(st);
    for (int r = 0; r < R; ++r)
      for (int k = 0; k < Ns; ++k) {
        const double a = -2.0 * M_PI * (double)(r * k) / (double)(Ns * R);
        h[Sh::twoff(st) + r * Ns + k] = C<T>{(T)std::cos(a), (T)std::sin(a)};
      }
  }
  return h;
}

constexpr int kGuard = 64;
const float kSentinel = 12345.0f;

template <typename Sh, int DIR, typename T, bool REG>
void check_shape(const char* name, std::mt19937_64& rng) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  static_assert(pad_linear<Sh>() || N > 0, "");
  const std::vector<C<T>> tw = twiddles<Sh, T>();
  std::normal_distribution<double> nd;
  std::vector<C<T>> x(N), out(N);
  for (auto& e : x) e = C<T>{(T)nd(rng), (T)nd(rng)};
  std::vector<C<T>> buf(LL + 2 * kGuard, C<T>{(T)kSentinel, (T)kSentinel});
  C<T>* line = buf.data() + kGuard;
  std::barrier<> bar(TPL);
  auto sync = [&bar] { bar.arrive_and_wait(); };
  std::vector<std::thread> lanes;
  lanes.reserve(TPL);
  for (int t = 0; t < TPL; ++t)
    lanes.emplace_back([&, t] {
      C<T> v[E];
      for (int m = 0; m < E; ++m) v[m] = x[t + TPL * m];
      if constexpr (REG) {
        TwReg<Sh, T> r;
        r.load(tw.data(), t);
        line_fft_tw<Sh, DIR, T>(v, t, line, r, sync);
      } else {
        line_fft<Sh, DIR, T>(v, t, line, tw.data(), sync);
      }
      for (int m = 0; m < E; ++m) out[t + TPL * m] = v[m];
    });
  for (auto& l : lanes) l.join();
  for (int i = 0; i < kGuard; ++i) {
    CHECK(buf[i].x == (T)kSentinel && buf[i].y == (T)kSentinel, "%s: write below the line", name);
    CHECK(buf[kGuard + LL + i].x == (T)kSentinel, "%s: write past the line", name);
  }
  // direct DFT in long double
  long double err = 0, rms = 0;
  for (int k = 0; k < N; ++k) {
    std::complex<long double> s = 0;
    for (int n = 0; n < N; ++n) {
      const long double a = (long double)DIR * 2.0L * 3.14159265358979323846264338327950288L *
                            (long double)((int64_t)k * n % N) / (long double)N;
      s += std::complex<long double>(x[n].x, x[n].y) * std::complex<long double>(std::cos(a), std::sin(a));
    }
    rms += std::norm(s);
    err = std::max(err, std::abs(s - std::complex<long double>(out[k].x, out[k].y)));
  }
  rms = std::sqrt(rms / N);
  const double rel = (double)(err / rms);
  const double bar_rel = sizeof(T) == 4 ? 3e-6 : 1e-14;
  std::printf("  %-34s DIR %+d %s %s  max err / rms = %.2e\n", name, DIR, sizeof(T) == 4 ? "fp32" : "fp64",
              REG ? "reg" : "lds", rel);
  CHECK(rel < bar_rel, "%s: error %.3e", name, rel);
}

template <typename Sh, typename T>
void check_all(const char* name, std::mt19937_64& rng) {
  check_shape<Sh, -1, T, false>(name, rng);
  check_shape<Sh, 1, T, false>(name, rng);
  if constexpr (Sh::E <= 8) {
    check_shape<Sh, -1, T, true>(name, rng);
    check_shape<Sh, 1, T, true>(name, rng);
  }
}

int main() {
  std::mt19937_64 rng(2024);
  check_all<DefaultShape<float, 64>::type, float>("Shape<64,2,8,8,1>", rng);
  check_all<DefaultShape<float, 128>::type, float>("Shape<128,3,8,8,2>", rng);
  check_all<DefaultShape<float, 256>::type, float>("Shape<256,3,8,8,4>", rng);
  check_all<DefaultShape<float, 512>::type, float>("Shape<512,3,8,8,8>", rng);
  check_all<DefaultShape<float, 1024>::type, float>("Shape<1024,3,16,8,8>", rng);
  check_all<AltShape<float, 64>::type, float>("Shape<64,2,16,4,1>", rng);
  check_all<AltShape<float, 128>::type, float>("Shape<128,2,16,8,1>", rng);
  check_all<AltShape<float, 256>::type, float>("Shape<256,2,16,16,1>", rng);
  check_all<AltShape<float, 512>::type, float>("Shape<512,3,16,8,4>", rng);
  check_all<AltShape<float, 1024>::type, float>("Shape<1024,3,16,16,4>", rng);
  check_all<DefaultShape<double, 64>::type, double>("Shape<64,2,8,8,1>", rng);
  check_all<DefaultShape<double, 256>::type, double>("Shape<256,3,8,8,4>", rng);
  check_all<DefaultShape<double, 1024>::type, double>("Shape<1024,3,16,8,8>", rng);
  check_all<DefaultShape<double, 512>::type, double>("Shape<512,3,8,8,8>", rng);
  std::printf("line transform checks passed\n");
  return 0;
}
