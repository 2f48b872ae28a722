// Host stand-in for the library calls serve.cpp makes (the step itself): a context over
// the caller's workspace; mpm_step flushes the stream's queued copies (stream order), then
// writes the particles back reversed, as a step writes them back in cell order, and
// exposes that permutation.
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstring>
#include <vector>
#include "mpm.h"
struct mpm_ctx { mpm_params p; char* ws; size_t bytes; int64_t cap_part, cap_surf; int32_t* perm; char* mirror; mpm_stats st; };
extern "C" {
int mpm_workspace_bytes(const mpm_params* p, int64_t cp, int64_t cs, size_t* out) {
  *out = 4096 + (size_t)cp * 4 + (size_t)(p->n) * 16; return MPM_OK; }
int mpm_ctx_create(const mpm_params* p, void* ws, size_t bytes, int64_t cp, int64_t cs, mpm_ctx** out) {
  size_t need; mpm_workspace_bytes(p, cp, cs, &need);
  if (!ws || bytes < need) return MPM_EINVAL;
  mpm_ctx* c = new mpm_ctx{*p, (char*)ws, bytes, cp, cs, (int32_t*)((char*)ws + 4096), nullptr, {}};
  hipHostMalloc((void**)&c->mirror, 1024, 0);
  std::memset(ws, 0, need);
  *out = c; return MPM_OK; }
int mpm_ctx_destroy(mpm_ctx* c) { hipHostFree(c->mirror); delete c; return MPM_OK; }
int mpm_step(mpm_ctx* const* cs, mpm_particles* const* P, const mpm_surface* const* S, int32_t n, int32_t, void* s) {
  hipStreamSynchronize((hipStream_t)s);
  for (int k = 0; k < n; ++k) {
    mpm_ctx* c = cs[k]; const int64_t N = P[k]->n; const int dim = c->p.dim;
    if (N > c->cap_part || S[k]->n > c->cap_surf) return MPM_ENOMEM;
    const bool f64 = c->p.precision == MPM_FP64; const size_t R = f64 ? 8 : 4;
    // read every surface sample and label the step would read
    volatile double acc = 0;
    for (int64_t i = 0; i < S[k]->n; ++i) acc += S[k]->label[i];
    void* f[8] = {P[k]->x, P[k]->v, P[k]->A, P[k]->J, P[k]->V0, P[k]->m, P[k]->T, P[k]->gradT};
    int nc[8] = {dim, dim, dim * dim, 1, 1, 1, 1, dim};
    std::vector<char> tmp;
    for (int q = 0; q < 8; ++q)
      for (int a = 0; a < nc[q]; ++a) {
        char* base = (char*)f[q] + (size_t)a * N * R;
        tmp.assign(base, base + N * R);
        for (int64_t i = 0; i < N; ++i) std::memcpy(base + i * R, tmp.data() + (N - 1 - i) * R, R);
      }
    for (int64_t i = 0; i < N; ++i) c->perm[i] = (int32_t)(N - 1 - i);
    c->st = mpm_stats{}; c->st.newton_iters = 1; c->st.n_part = N; c->st.n_surf = S[k]->n;
  }
  return MPM_OK; }
// The device sampler: the host stage on the (host-resident) positions, written out in the
// device layout [dim][count] of the context's real type.
int mpm_sample_surface_dev(mpm_ctx* c, const mpm_particles* P, double radius, double density, uint64_t seed,
                           uint64_t step, const double* lo, const double* hi, void* s_out, void* dA_out,
                           int32_t* label, int64_t cap, int64_t* out_n, void* s) {
  hipStreamSynchronize((hipStream_t)s);
  const int dim = c->p.dim; const int64_t N = P->n; const bool f64 = c->p.precision == MPM_FP64;
  std::vector<double> x((size_t)dim * N);
  for (size_t i = 0; i < x.size(); ++i) x[i] = f64 ? ((const double*)P->x)[i] : ((const float*)P->x)[i];
  int64_t hcap = 4 * N + 4096, cnt = 0;
  std::vector<double> hs, hdA;
  std::vector<int32_t> hl;
  for (;;) {
    hs.assign((size_t)dim * hcap, 0.0); hdA.assign((size_t)dim * hcap, 0.0); hl.assign(hcap, 0);
    int rc = mpm_sample_surface(dim, c->p.n, x.data(), N, radius, density, seed, step, lo, hi, hs.data(), hdA.data(),
                                hl.data(), hcap, &cnt);
    if (rc != MPM_OK) return rc;
    if (cnt <= hcap) break;
    hcap = cnt;
  }
  *out_n = cnt;
  if (cnt > cap) return MPM_OK;
  for (int a = 0; a < dim; ++a)
    for (int64_t i = 0; i < cnt; ++i) {
      if (f64) { ((double*)s_out)[a * cnt + i] = hs[a * hcap + i]; ((double*)dA_out)[a * cnt + i] = hdA[a * hcap + i]; }
      else { ((float*)s_out)[a * cnt + i] = (float)hs[a * hcap + i]; ((float*)dA_out)[a * cnt + i] = (float)hdA[a * hcap + i]; }
    }
  if (label) std::memcpy(label, hl.data(), cnt * 4);
  return MPM_OK;
}
int mpm_get_stats(const mpm_ctx* c, mpm_stats* o) { *o = c->st; return MPM_OK; }
int mpm_grid_view(mpm_ctx* c, int32_t f, void** out) { if (f != MPM_F_PERM) return MPM_EINVAL; *out = c->perm; return MPM_OK; }
}
extern "C" int mpm_params_default(mpm_params* p, int32_t dim, int32_t n) {
  std::memset(p, 0, sizeof(*p)); p->dim = dim; p->n = n; p->dx = 1.0 / n; p->dt = 1e-3; return MPM_OK; }
