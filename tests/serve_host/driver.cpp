// Serving stream through the serving runtime with the host stand-ins: 8 workers, droplets
// on n in {16, 32, 48, 64} and every tenth request a sparse cloud that outgrows its first
// surface sizing, every request borrowing its host arrays, results checked against the
// reversal the stand-in step applies (twice per two steps).
#include <cmath>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>
#include "mpm.h"
int main(int argc, char** argv) {
  const int nreq = argc > 1 ? atoi(argv[1]) : 200, workers = 8;
  std::vector<char> arena((size_t)1 << 30);
  char* base = (char*)(((uintptr_t)arena.data() + 255) & ~(uintptr_t)255);
  mpm_server* srv = nullptr;
  if (mpm_server_create(base, (size_t)768 << 20, workers, &srv) != MPM_OK) return 2;
  std::mt19937_64 rng(5);
  const int sizes[4] = {16, 32, 48, 64};
  struct Host { std::vector<double> f[8]; int64_t N; int steps; };
  std::vector<Host> hs(nreq);
  for (int r = 0; r < nreq; ++r) {
    const int n = sizes[rng() % 4]; const double dx = 1.0 / n, rad = 0.24;
    std::vector<double> pts;
    if (r % 10 == 7) {
      // a sparse cloud: every particle its own sphere, far more samples than particles,
      // so the request outgrows its first sizing and is queued again
      std::uniform_real_distribution<double> u(0.2, 0.8);
      for (int p = 0; p < 150; ++p) { double x[3] = {u(rng), u(rng), u(rng)}; pts.insert(pts.end(), x, x + 3); }
    } else {
      for (int k = 0; k < n; ++k) for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i)
        for (int s = 0; s < 8; ++s) {
          double x[3] = {(i + 0.25 + 0.5 * (s & 1)) * dx, (j + 0.25 + 0.5 * ((s >> 1) & 1)) * dx, (k + 0.25 + 0.5 * (s >> 2)) * dx};
          double d2 = 0; for (double t : x) d2 += (t - 0.5) * (t - 0.5);
          if (d2 < rad * rad) pts.insert(pts.end(), x, x + 3);
        }
    }
    Host& h = hs[r]; h.N = (int64_t)pts.size() / 3; h.steps = 1 + (int)(rng() % 2);
    const int nc[8] = {3, 3, 9, 1, 1, 1, 1, 3};
    for (int q = 0; q < 8; ++q) h.f[q].assign((size_t)nc[q] * h.N, 0.0);
    for (int64_t p = 0; p < h.N; ++p) for (int a = 0; a < 3; ++a) h.f[0][a * h.N + p] = pts[3 * p + a];
    for (int64_t p = 0; p < h.N; ++p) { h.f[1][p] = p; h.f[3][p] = 1; h.f[4][p] = dx * dx * dx / 8; h.f[5][p] = 1; h.f[6][p] = 300 + p; }
    mpm_request q{}; mpm_params_default(&q.params, 3, n);
    q.params.precision = (r % 3 == 0) ? MPM_FP64 : MPM_MIXED;
    q.id = r; q.n_steps = h.steps; q.implicit = 1; q.keep_result = 1; q.borrow = 1; q.n_part = h.N; q.seed = 1000 + r;
    q.x = h.f[0].data(); q.v = h.f[1].data(); q.A = h.f[2].data(); q.J = h.f[3].data(); q.V0 = h.f[4].data();
    q.m = h.f[5].data(); q.T = h.f[6].data(); q.gradT = h.f[7].data();
    if (mpm_server_submit(srv, &q) != MPM_OK) return 3;
  }
  if (mpm_server_wait(srv, -1.0) != MPM_OK) return 4;
  int bad = 0;
  for (int r = 0; r < nreq; ++r) {
    Host& h = hs[r]; std::vector<double> x(3 * h.N), v(3 * h.N), A(9 * h.N), J(h.N), T(h.N), g(3 * h.N);
    int st = mpm_server_result(srv, r, x.data(), v.data(), A.data(), J.data(), T.data(), g.data());
    if (st != MPM_OK) { ++bad; continue; }
    // results come back in request order: the stand-in's reversal is undone by the server
    for (int64_t p = 0; p < h.N; ++p)
      if (std::fabs(v[p] - (double)p) > 0.5 || std::fabs(T[p] - (300.0 + p)) > 0.5 * (300.0 + p) * 1e-6 + 0.5) { ++bad; break; }
  }
  mpm_server_info info{}; mpm_server_info_get(srv, &info);
  mpm_server_destroy(srv);
  std::printf("requests %d, bad %d, peak running %d, peak bytes %lld\n", nreq, bad, info.peak_running, (long long)info.peak_bytes);
  return bad ? 1 : 0;
}
