// Host side of the MPM hot-path library: workspace layout, contexts, the step pipeline
// and the C ABI declared in include/mpm.h.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tiles.h"
#include "sampler_dev.h"

using namespace mpm;

// Scratch of mpm_step_noalloc (see there): the largest workspace it can carve.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kNumParts = 20;   // partial-sum slots: momentum 0..15 (merge: D+5 from slot 4; correction: 2D+4 from 0), heat 16..19
constexpr int kScalDoubles = 64;
// Device scalars the host reads back, in one block so that every read is one copy:
// [0, 512) FP64 scalar slots, [512, 672) the two CG scalar sets, [768, 1024) status words.
constexpr int kMirrorBytes = 1024, kMirrorCg = 512, kMirrorMisc = 768, kMirrorRead = 800;
// Host-only slot of the pinned mirror (past the part that read_mirror copies): the heat
// solve's CG scalars, read on their own stream.
constexpr int kMirrorHeatHost = 896;
// The CFL step's particle maxima (k_max_speed), behind the three CG scalar sets.
constexpr int kMirrorCfl = 752;

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) throw HipError{e_, #x};   \
  } while (0)

struct ApiError {
  int code;
  std::string msg;
};

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Bump allocator over the workspace (256-byte aligned pieces).
struct Bump {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace

// Per-kernel-class timing with HIP events stamped by the launches themselves.
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;      // pairs (start, stop)
  std::vector<int> cls;
  size_t used = 0;
  double ms[MPM_K_COUNT] = {};
  int64_t launches[MPM_K_COUNT] = {};
  std::vector<float> dur[MPM_K_COUNT];   // every launch's duration (ms)
};

struct mpm_ctx {
  mpm_params p;
  Prof prof;
  int dim = 3, n = 0, nt = 0, nn = 0, ntile_total = 0;
  int64_t cap_part = 0, cap_surf = 0;
  bool fp64 = true;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // typed device views (only the one matching the precision is used)
  Dev<double> d64{};
  Dev<float> d32{};
  // real-typed vectors (void* so both precisions share the host code)
  void *vhat = nullptr, *vtrial = nullptr, *grad = nullptr, *delta = nullptr, *r = nullptr, *z = nullptr,
       *pp = nullptr, *Ap = nullptr, *zero = nullptr, *gscratch = nullptr;
  // a second set of momentum-CG vectors (delta, r, z, p, Ap): Newton iterations alternate
  // sets, so that the next iteration's CG can be queued before the current one is judged
  void* cg2[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  void *That = nullptr, *hr = nullptr, *hz = nullptr, *hp = nullptr, *hAp = nullptr;
  int* tile_pos = nullptr;
  int* ctile_flag = nullptr;
  int* ctile_pos = nullptr;
  int* ctile_list = nullptr;
  int* ctile_slot = nullptr;
  int* ctile_rng = nullptr;
  int* nbr_slot = nullptr;
  void* tpart = nullptr;        // per-cell-tile region partials
  void* tpart_heat = nullptr;   // the heat operator's (separate: it may run concurrently)
  int nctile = 0;
  uint64_t* scan_flags = nullptr;   // status words of the single-pass scan (kScanBlock)
  unsigned scan_epoch = 0;
  // the same sort scratch for the surface-sample sort on the second stream
  int* ccount_aux = nullptr;
  int* sort_tmp_aux = nullptr;
  void* sF_alt = nullptr;        // surface F_r at the line-search trial (swapped with d.sF)
  // device surface sampler: its own particle binning and the dense node / cube arrays
  int *smp_key = nullptr, *smp_perm = nullptr, *smp_start = nullptr, *smp_cnt = nullptr, *smp_off = nullptr;
  uint8_t* smp_flag = nullptr;
  double* smp_phi = nullptr;
  uint64_t* scan_flags_aux = nullptr;
  unsigned scan_epoch_aux = 0;
  int* misc = nullptr;          // [0] status, [1] constrained flag, [2] tile count
  double* part = nullptr;
  double* scal = nullptr;
  CgScal* cg = nullptr;
  unsigned* ctr = nullptr;       // grid-reduction counters
  int* sort_tmp = nullptr;       // segment-order scratch (max(cap_part, cap_surf) ints)
  // pinned host mirror of the device scalar block (hbuf, hcg, hint point into it)
  char* hmirror = nullptr;
  double* hbuf = nullptr;
  int* hint = nullptr;
  CgScal* hcg = nullptr;
  // state
  int np = 0, ns = 0, ntiles = 0, prev_ntiles = 0, prev_nctile = 0;
  bool have_p2g = false, constrained = false, mom_pending = false;
  // Krylov launch schedule learned from the previous solves (first chunk sizes)
  int cg_hint_mom = 2, cg_hint_heat = 2;
  // run lengths of the tile kernels' XCD slot mapping picked by mpm_autotune (energy,
  // Hessian, heat; 0: the size heuristic xcd_run)
  int run_tuned[3] = {0, 0, 0};
  int status = 0;
  mpm_stats stats{};
  std::string err;
  // batch execution: the device the context lives on, its own stream and done event
  int device = 0;
  hipStream_t own = nullptr;
  hipEvent_t own_done = nullptr;
  // second stream of a step: the heat solve runs beside the momentum solve
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_hread = nullptr, ev_counts = nullptr, ev_sfork = nullptr,
             ev_sjoin = nullptr, ev_mread = nullptr;
  // single-stream mode (the context of mpm_step_noalloc): every chain runs on the caller's
  // stream and the host waits on that stream, so no stream or event is ever created
  bool single = false;
  hipStream_t mread_stream = nullptr;
};

namespace {

// The start and stop events of the next timed launch.  They are given to the launch
// itself (hipExtLaunchKernelGGL), which stamps them with the kernel's own begin and end,
// so the elapsed time is the kernel's, without the time of separate event markers.
void prof_slot(mpm_ctx* c, int cls, hipEvent_t* start, hipEvent_t* stop) {
  Prof& pr = c->prof;
  if (pr.used * 2 + 2 > pr.ev.size()) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    pr.ev.push_back(a);
    pr.ev.push_back(b);
    pr.cls.push_back(0);
  }
  pr.cls[pr.used] = cls;
  *start = pr.ev[2 * pr.used];
  *stop = pr.ev[2 * pr.used + 1];
  pr.used++;
}

void prof_collect(mpm_ctx* c) {
  Prof& pr = c->prof;
  for (size_t k = 0; k < pr.used; ++k) {
    HIPCHK(hipEventSynchronize(pr.ev[2 * k + 1]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, pr.ev[2 * k], pr.ev[2 * k + 1]));
    pr.ms[pr.cls[k]] += ms;
    pr.launches[pr.cls[k]] += 1;
    pr.dur[pr.cls[k]].push_back(ms);
  }
  pr.used = 0;
}

// Launches of class k that did work: a CG called off on the device still launches its
// kernels, which return at once.  Those below a tenth of the class's 95th-percentile
// duration are left out.
void prof_work(const Prof& pr, int k, double* ms, int64_t* n) {
  std::vector<float> v = pr.dur[k];
  *ms = 0;
  *n = 0;
  if (v.empty()) return;
  std::sort(v.begin(), v.end());
  const double p95 = v[(size_t)std::floor(0.95 * (double)(v.size() - 1))];
  for (float x : v)
    if (x >= 0.1 * p95) { *ms += x; ++*n; }
}

// Launch on stream s (in scope), timed as kernel class cls when timing is on.
#define LAUNCH(c, cls, K, G, B, SH, S, ...)                                   \
  do {                                                                        \
    if ((c)->prof.on) {                                                       \
      hipEvent_t start_, stop_;                                               \
      prof_slot((c), (cls), &start_, &stop_);                                 \
      hipExtLaunchKernelGGL(K, G, B, SH, S, start_, stop_, 0, ##__VA_ARGS__); \
    } else {                                                                  \
      hipLaunchKernelGGL(K, G, B, SH, S, ##__VA_ARGS__);                      \
    }                                                                         \
  } while (0)

inline bool solids_on(const mpm_params& p) { return p.T_melt > -1e299; }

template <typename R>
size_t layout(mpm_ctx* c, char* base) {
  Bump b{base};
  const int D = c->dim;
  const int64_t NP = std::max<int64_t>(c->cap_part, 1), NS = std::max<int64_t>(c->cap_surf, 1);
  const int64_t NN = c->nn, NT = c->ntile_total;
  Dev<R> d{};
  d.p_start = b.take<int>(NN + 1); d.p_perm = b.take<int>(NP); d.p_key = b.take<int>(NP);
  d.pcnt = b.take<int>(NP); d.pcnt_orig = b.take<int>(NP); d.grp_start = b.take<int>(NP + 1); d.grp = b.take<int>(NS); d.gcur = b.take<int>(NP);
  d.s_start = b.take<int>(NN + 1); d.s_perm = b.take<int>(NS); d.s_key = b.take<int>(NS);
  d.slabel = b.take<int>(NS); d.spar = b.take<int>(NS); d.s_parent_orig = b.take<int>(NS);
  d.b_start = b.take<int>(NN + 1); d.b_src = b.take<int>(NS); d.b_key = b.take<int>(NS);
  d.ccount = b.take<int>(NN);
  d.tile_flag = b.take<int>(NT); d.tile_list = b.take<int>(NT);
  int* tile_pos = b.take<int>(NT + 1);
  int* ctile_flag = b.take<int>(2 * NT);
  int* ctile_pos = b.take<int>(2 * NT + 1);
  int* ctile_list = b.take<int>(NT);
  int* ctile_slot = b.take<int>(NT);
  int* ctile_rng = b.take<int>(6 * NT);
  int* nbr_slot = b.take<int>((size_t)kNbr * NT);
  const int64_t nct_cap = std::min<int64_t>(NT, NP + 2 * NS);
  const int RNd = D == 3 ? TileGeo<3>::RN : TileGeo<2>::RN;
  const int NFmax = std::max(2 * D + 7, D);
  void* tpart = b.take<R>((size_t)nct_cap * RNd * NFmax);
  void* tpart_heat = b.take<R>((size_t)nct_cap * RNd);
  uint64_t* scan_flags = b.take<uint64_t>(kScanBlock);
  char* mirror = b.take<char>(kMirrorBytes);
  int* misc = (int*)(mirror + kMirrorMisc);
  d.px = b.take<R>(D * NP); d.pv = b.take<R>(D * NP); d.pA = b.take<R>(D * D * NP);
  d.pm = b.take<R>(NP); d.pmt = b.take<R>(NP); d.pJ = b.take<R>(NP); d.pV0 = b.take<R>(NP);
  d.pT = b.take<R>(NP); d.pgT = b.take<R>(D * NP); d.pmu = b.take<R>(NP); d.pVn = b.take<R>(NP);
  d.pHc = b.take<R>(2 * NP);
  d.ss = b.take<R>(D * NS); d.sdA = b.take<R>(D * NS); d.sk = b.take<R>(NS); d.sk_orig = b.take<R>(NS);
  const bool sol = solids_on(c->p);
  const int64_t NL = NS + (sol ? NP : 0);   // linearization cache: surface samples, then solid particles
  d.sc = b.take<R>((D + D * D) * NS); d.sF = b.take<R>(D * D * NL); d.bx = b.take<R>(D * NS); d.bx_unsorted = b.take<R>(D * NS);
  d.solids = sol ? 1 : 0;
  d.pF = sol ? b.take<R>(D * D * NP) : nullptr;
  d.pSol = sol ? b.take<R>(NP) : nullptr;
  d.pLh = sol ? b.take<R>(2 * NP) : nullptr;
  d.gm = b.take<R>(NN); d.gW = b.take<R>(NN); d.gWT = b.take<R>(NN); d.gE = b.take<R>(NN);
  d.gET = b.take<R>(NN); d.gTn = b.take<R>(NN); d.hdiag = b.take<R>(NN); d.hrhs = b.take<R>(NN);
  d.gmv = b.take<R>(D * NN); d.gvn = b.take<R>(D * NN); d.gdiag = b.take<R>(D * NN);
  d.gfree = b.take<uint8_t>(NN);
  void* vecs[15];
  for (int k = 0; k < 15; ++k) vecs[k] = b.take<R>(D * NN);
  void* hvecs[5];
  for (int k = 0; k < 5; ++k) hvecs[k] = b.take<R>(NN);
  d.part = b.take<double>((size_t)kNumParts * kPartSlot);
  d.scal = (double*)mirror;
  CgScal* cg = (CgScal*)(mirror + kMirrorCg);
  static_assert(kScalDoubles * sizeof(double) <= kMirrorCg && kMirrorCg + 3 * sizeof(CgScal) <= kMirrorMisc &&
                    kMirrorCg + 3 * sizeof(CgScal) <= kMirrorCfl && kMirrorCfl + 16 <= kMirrorMisc &&
                    kMirrorMisc + 8 * sizeof(int) <= kMirrorRead && kMirrorRead <= kMirrorHeatHost &&
                    kMirrorHeatHost + sizeof(CgScal) <= kMirrorBytes,
                "mirror layout");
  unsigned* ctr = b.take<unsigned>((size_t)CTR_COUNT * kCtrSite);
  int* sort_tmp = b.take<int>(std::max(NP, NS));
  int* ccount_aux = b.take<int>(NN);
  int* sort_tmp_aux = b.take<int>(NS);
  void* sF_alt = b.take<R>(D * D * NL);
  uint64_t* scan_flags_aux = b.take<uint64_t>(kScanBlock);
  int* smp_key = b.take<int>(NP);
  int* smp_perm = b.take<int>(NP);
  int* smp_start = b.take<int>(NN + 1);
  int* smp_cnt = b.take<int>(NN);
  int* smp_off = b.take<int>(NN + 1);
  uint8_t* smp_flag = b.take<uint8_t>(NN);
  double* smp_phi = b.take<double>(NN);
  d.status = misc;
  if (base) {
    c->vhat = vecs[0]; c->vtrial = vecs[1]; c->grad = vecs[2]; c->delta = vecs[3]; c->r = vecs[4];
    c->z = vecs[5]; c->pp = vecs[6]; c->Ap = vecs[7]; c->zero = vecs[8]; c->gscratch = vecs[9];
    for (int k = 0; k < 5; ++k) c->cg2[k] = vecs[10 + k];
    c->That = hvecs[0]; c->hr = hvecs[1]; c->hz = hvecs[2]; c->hp = hvecs[3]; c->hAp = hvecs[4];
    c->tile_pos = tile_pos; c->scan_flags = scan_flags; c->misc = misc;
    c->ctile_flag = ctile_flag; c->ctile_pos = ctile_pos; c->ctile_list = ctile_list; c->ctile_slot = ctile_slot;
    c->ctile_rng = ctile_rng;
    c->nbr_slot = nbr_slot;
    c->tpart = tpart;
    c->tpart_heat = tpart_heat;
    c->part = d.part; c->scal = d.scal; c->cg = cg; c->ctr = ctr;
    c->sort_tmp = sort_tmp;
    c->ccount_aux = ccount_aux; c->sort_tmp_aux = sort_tmp_aux; c->scan_flags_aux = scan_flags_aux;
    c->sF_alt = sF_alt;
    c->smp_key = smp_key; c->smp_perm = smp_perm; c->smp_start = smp_start; c->smp_cnt = smp_cnt;
    c->smp_off = smp_off; c->smp_flag = smp_flag; c->smp_phi = smp_phi;
    if constexpr (sizeof(R) == 8) c->d64 = d; else c->d32 = d;
  }
  return b.off + 256;
}

template <typename R>
void fill_params(Dev<R>& d, const mpm_params& p, int nt) {
  d.n = p.n; d.nt = nt; d.nn = 1;
  for (int a = 0; a < p.dim; ++a) d.nn *= p.n;
  d.fn = (R)p.n; d.dx = (R)p.dx; d.dt = (R)p.dt;
  d.lam = (R)p.bulk; d.mu0 = (R)p.mu0; d.mu_k = (R)p.mu_k; d.mu_T0 = (R)p.mu_T0;
  d.g0 = (R)p.g0; d.g1 = (R)p.g1; d.gT0 = (R)p.gT0; d.gmin = (R)p.gmin; d.gmax = (R)p.gmax;
  d.cp = (R)p.cp; d.K = (R)p.K; d.h = (R)p.h; d.T_amb = (R)p.T_amb; d.b = (R)p.b; d.H = (R)p.H;
  for (int k = 0; k < 4; ++k) d.gamma_label[k] = (R)p.gamma_label[k];
  for (int k = 0; k < 3; ++k) {
    d.grav[k] = (R)p.gravity[k]; d.slab_lo[k] = (R)p.slab_lo[k]; d.slab_hi[k] = (R)p.slab_hi[k];
  }
  d.slab = p.slab; d.slab_axis = p.slab_axis; d.wall = p.wall_layers; d.term_mask = p.term_mask;
  d.exact = p.hess_mode == MPM_HESS_EXACT; d.gamma_by_label = p.gamma_by_label;
  d.T_melt = p.T_melt; d.muh0 = (R)p.muh0; d.lamh0 = (R)p.lamh0; d.kh = (R)p.kh; d.Th0 = (R)p.Th0;
}

void check_params(const mpm_params* p) {
  if (!p) throw ApiError{MPM_EINVAL, "null params"};
  if (p->dim != 2 && p->dim != 3) throw ApiError{MPM_EINVAL, "dim must be 2 or 3"};
  if (p->n < 8 || p->n % 8 != 0) throw ApiError{MPM_EINVAL, "n must be a positive multiple of 8"};
  double nn = std::pow((double)p->n, p->dim);
  if (nn > (double)(kScanBlock) * kScanBlock) throw ApiError{MPM_EINVAL, "n^dim above 2^24"};
  if (!(std::fabs(p->dx * p->n - 1.0) < 1e-9)) throw ApiError{MPM_EINVAL, "dx must equal 1/n"};
  if (!(p->dt > 0)) throw ApiError{MPM_EINVAL, "dt must be positive"};
  if (p->precision != MPM_FP64 && p->precision != MPM_MIXED) throw ApiError{MPM_EINVAL, "bad precision"};
  if (p->slab_axis < 0 || p->slab_axis >= p->dim) throw ApiError{MPM_EINVAL, "bad slab_axis"};
  if (p->krylov != MPM_KRYLOV_CG && p->krylov != MPM_KRYLOV_MINRES) throw ApiError{MPM_EINVAL, "bad krylov"};
  if (p->gamma_by_label < 0 || p->gamma_by_label > 2) throw ApiError{MPM_EINVAL, "gamma_by_label must be 0, 1 or 2"};
  if (p->n_planes < 0 || p->n_planes > MPM_MAX_PLANES) throw ApiError{MPM_EINVAL, "n_planes must be in [0, 4]"};
  if (p->T_melt > -1e299 && p->hess_mode == MPM_HESS_EXACT)
    throw ApiError{MPM_EINVAL, "hess_mode EXACT is not available with solids (T_melt set)"};
  for (int k = 0; k < p->n_planes; ++k) {
    double l2 = 0;
    for (int a = 0; a < 3; ++a) l2 += p->plane_n[k][a] * p->plane_n[k][a];
    if (!(std::fabs(l2 - 1.0) < 1e-9)) throw ApiError{MPM_EINVAL, "plane_n must be unit normals"};
    if (!(p->plane_mu[k] >= 0)) throw ApiError{MPM_EINVAL, "plane_mu must be >= 0"};
  }
}

// Scratch of one cell sort: cell counters (zero between sorts), the scan's status words
// with their epoch, segment-order scratch.  The surface-sample sort runs on the second
// stream beside the particle sort with a set of its own.
struct SortRes {
  int* ccount;
  uint64_t* flags;
  unsigned* epoch;
  int* tmp;
};
template <typename R>
SortRes sort_res(mpm_ctx* c, Dev<R>& d, bool aux) {
  return aux ? SortRes{c->ccount_aux, c->scan_flags_aux, &c->scan_epoch_aux, c->sort_tmp_aux}
             : SortRes{d.ccount, c->scan_flags, &c->scan_epoch, c->sort_tmp};
}

// ---- exclusive scan of len ints: out[0..len) and out[len] = total ----------------------
void scan(mpm_ctx* c, const int* in, int* out, int len, hipStream_t s, uint64_t* flags, unsigned* epoch) {
  int nb = cdiv(len, kScanBlock);
  if (nb > kScanBlock) throw ApiError{MPM_EINVAL, "scan length above 2^24"};
  if (((uintptr_t)in | (uintptr_t)out) % 16) throw ApiError{MPM_EINVAL, "scan buffers not 16-byte aligned"};
  if (len == 0) {
    LAUNCH(c, MPM_K_SORT, k_fill_i32, dim3(1), dim3(1), 0, s, out, 0, (int64_t)1);
    return;
  }
  // the status words of one scan are told from older ones by the epoch (never 0, the
  // value of the zeroed workspace)
  *epoch = *epoch % ((1u << 30) - 1) + 1;
  LAUNCH(c, MPM_K_SORT, k_scan, dim3(nb), dim3(kScanT), 0, s, in, out, len, flags, *epoch, c->misc);
}
void scan(mpm_ctx* c, const int* in, int* out, int len, hipStream_t s) {
  scan(c, in, out, len, s, c->scan_flags, &c->scan_epoch);
}

// Copies src[0, cnt) to dst with every segment (run of equal key[value], starting at
// start[key]) in ascending value order.
void segment_order(mpm_ctx* c, const int* key, const int* start, int cnt, const int* src, int* dst, hipStream_t s) {
  if (cnt <= 0) return;
  LAUNCH(c, MPM_K_SORT, k_segment_order, dim3(cdiv(cnt, 256)), dim3(256), 0, s, key, start, cnt, src, dst);
}

// Stable cell sort of cnt points: perm (sorted slot -> input index) and start[nn+1].
// Dense cell counts give the cell starts; an atomic scatter places the points, and each
// cell's segment is then put in input order, so the result does not depend on the order
// in which the atomics were served.
// counted: keys and counts are already in key and r.ccount.
template <int D, typename R>
void cell_sort(mpm_ctx* c, Dev<R>& d, const R* pos, int cnt, int* key, int* perm, int* start, hipStream_t s,
               const SortRes& r, bool counted = false) {
  if (cnt > 0 && !counted)
    LAUNCH(c, MPM_K_SORT, (k_cell_keys<D, R>), dim3(cdiv(cnt, 256)), dim3(256), 0, s, pos, cnt, d.n, d.nt, d.fn, key,
           r.ccount, d.status);
  scan(c, r.ccount, start, d.nn, s, r.flags, r.epoch);
  if (cnt > 0) {
    LAUNCH(c, MPM_K_SORT, k_cell_scatter, dim3(cdiv(cnt, 256)), dim3(256), 0, s, (const int*)key, cnt,
           (const int*)start, r.ccount, r.tmp, d.status);
    segment_order(c, key, start, cnt, (const int*)r.tmp, perm, s);
  }
}

template <typename R> Dev<R>& dev(mpm_ctx* c);
template <> Dev<double>& dev<double>(mpm_ctx* c) { return c->d64; }
template <> Dev<float>& dev<float>(mpm_ctx* c) { return c->d32; }

// Tile kernel classes whose XCD run length mpm_autotune picks.
enum : int { TUNE_ENERGY = 0, TUNE_HESS = 1, TUNE_HEAT = 2, TUNE_COUNT = 3 };
int run_for(const mpm_ctx* c, int k) { return c->run_tuned[k] > 0 ? c->run_tuned[k] : xcd_run(c->nctile); }

// Whether the energy evaluation caches a Hessian linearization (surface F_r, solid cof F_p).
template <typename R>
bool lin_cache(const Dev<R>& d) { return (d.term_mask & 2) || d.solids; }

// The stress kernel variant of a scene: with solids; the J term alone (no viscosity: the
// viscous term off, or mu0 = 0); else the full fluid.
template <typename R>
int stress_var(const Dev<R>& d) {
  if (d.solids) return SV_SOLID;
  return ((d.term_mask & 4) == 0 || d.mu0 == R(0)) ? SV_JONLY : SV_FLUID;
}

TileLists tiles(mpm_ctx* c, int k = TUNE_ENERGY) {
  TileLists t;
  t.ctile_list = c->ctile_list;
  t.ctile_slot = c->ctile_slot;
  t.ctile_rng = c->ctile_rng;
  t.nbr = c->nbr_slot;
  t.nctile = c->nctile;
  t.xrun = run_for(c, k);
  return t;
}
// Grid of a tile kernel that takes its slot with xcd_slot.
int tile_grid(const mpm_ctx* c, int k = TUNE_ENERGY) { return xcd_grid(c->nctile, run_for(c, k)); }

int krylov_blocks(int nelem) { return std::max(1, std::min(1024, cdiv(nelem, kNodeThreads))); }
int merge_blocks(const mpm_ctx* c) { return merge_grid(c->ntiles); }

void sync_read(mpm_ctx* c, hipStream_t s, const void* src, void* dst, size_t bytes) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c->stats.host_waits++;
}

// The second stream of a context, ordered after the work queued so far on s (the
// caller's stream itself in single-stream mode); aux_join orders s after the work queued
// since on the returned stream.  fork/join: the two event pairs of the binning and of the
// heat solve.
hipStream_t aux_fork(mpm_ctx* c, hipStream_t s, hipEvent_t* fork) {
  if (c->single) return s;
  if (!c->aux) HIPCHK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
  if (!*fork) HIPCHK(hipEventCreateWithFlags(fork, hipEventDisableTiming));
  HIPCHK(hipEventRecord(*fork, s));
  HIPCHK(hipStreamWaitEvent(c->aux, *fork, 0));
  return c->aux;
}
void aux_mark(mpm_ctx* c, hipStream_t a, hipEvent_t* join) {
  if (c->single) return;
  if (!*join) HIPCHK(hipEventCreateWithFlags(join, hipEventDisableTiming));
  HIPCHK(hipEventRecord(*join, a));
}
void aux_join(mpm_ctx* c, hipStream_t s, hipEvent_t join) {
  if (c->single) return;
  HIPCHK(hipStreamWaitEvent(s, join, 0));
}
// A host wait point on stream s: mark records it, wait blocks until s has reached it (in
// single-stream mode: until s is idle).
void host_mark(mpm_ctx* c, hipStream_t s, hipEvent_t* ev) {
  if (c->single) return;
  if (!*ev) HIPCHK(hipEventCreateWithFlags(ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(*ev, s));
}
void host_wait(mpm_ctx* c, hipStream_t s, hipEvent_t ev) {
  if (c->single) HIPCHK(hipStreamSynchronize(s));
  else HIPCHK(hipEventSynchronize(ev));
  c->stats.host_waits++;
}

// The second stream's share of the binning (on stream s): clears the previous step's
// tiles, then bins the surface samples by cell and stages them in cell order.
template <int D, typename R>
void front_aux(mpm_ctx* c, Dev<R>& d, const mpm_surface* S, hipStream_t s) {
  if (c->prev_ntiles > 0)
    LAUNCH(c, MPM_K_SETUP, (k_clear_tiles<D, R>), dim3(c->prev_ntiles), dim3(64), 0, s, d, (const int*)d.tile_list,
           (R* const*)nullptr, 0, 0);
  if (c->ns > 0) {
    cell_sort<D, R>(c, d, (const R*)S->s, c->ns, d.s_key, d.s_perm, d.s_start, s, sort_res(c, d, true));
    LAUNCH(c, MPM_K_SETUP, (k_gather_surface<D, R>), dim3(cdiv(c->ns, 256)), dim3(256), 0, s, d, (const R*)S->s,
           (const R*)S->dA, S->label);
  }
}

// Active node tiles (hold a stencil node of a point), compacted into the tile list, and
// the count copied to the host (on stream s).
template <int D, typename R>
void node_tiles(mpm_ctx* c, Dev<R>& d, hipStream_t s) {
  LAUNCH(c, MPM_K_SETUP, (k_mark_tiles<D, R>), dim3(cdiv(d.nn, 256)), dim3(256), 0, s, d);
  scan(c, d.tile_flag, c->tile_pos, c->ntile_total, s, c->scan_flags_aux, &c->scan_epoch_aux);
  LAUNCH(c, MPM_K_SETUP, k_compact_tiles, dim3(cdiv(c->ntile_total, 256)), dim3(256), 0, s, (const int*)d.tile_flag,
         (const int*)c->tile_pos, c->ntile_total, d.tile_list);
  HIPCHK(hipMemcpyAsync(c->hint, c->tile_pos + c->ntile_total, sizeof(int), hipMemcpyDeviceToHost, s));
}

// ---------------------------------------------------------------------------------------
template <int D, typename R>
void do_p2g(mpm_ctx* c, const mpm_particles* P, const mpm_surface* S, hipStream_t s) {
  if (!P || P->n < 0 || P->n > c->cap_part) throw ApiError{MPM_ENOMEM, "particle count above capacity"};
  int64_t ns = S ? S->n : 0;
  if (ns < 0 || ns > c->cap_surf) throw ApiError{MPM_ENOMEM, "surface count above capacity"};
  if (P->n > 0 && (!P->x || !P->v || !P->A || !P->J || !P->V0 || !P->m || !P->T || !P->gradT))
    throw ApiError{MPM_EINVAL, "null particle buffer"};
  if (ns > 0 && (!S->s || !S->dA)) throw ApiError{MPM_EINVAL, "null surface buffer"};
  if (ns > 0 && P->n == 0) throw ApiError{MPM_EINVAL, "surface samples without particles"};
  Dev<R>& d = dev<R>(c);
  if (d.solids && P->n > 0 && !P->F) throw ApiError{MPM_EINVAL, "particles need F when T_melt is set"};
  c->np = (int)P->n;
  c->ns = (int)ns;
  d.np = c->np;
  d.ns = c->ns;
  LAUNCH(c, MPM_K_SORT, k_fill_i32, dim3(1), dim3(64), 0, s, c->misc, 0, (int64_t)8);
  // Independent chains go to the second stream: the clearing of the previous step's
  // tiles (views read zero outside the new active set) and the binning of the surface
  // samples, beside the binning of the interior particles on this stream.
  hipStream_t a = aux_fork(c, s, &c->ev_sfork);
  front_aux<D, R>(c, d, S, a);
  aux_mark(c, a, &c->ev_sjoin);
  cell_sort<D, R>(c, d, (const R*)P->x, c->np, d.p_key, d.p_perm, d.p_start, s, sort_res(c, d, false));
  if (c->np > 0)
    LAUNCH(c, MPM_K_SETUP, (k_gather_particles<D, R>), dim3(cdiv(c->np, 256)), dim3(256), 0, s, d, (const R*)P->x,
                       (const R*)P->v, (const R*)P->A, (const R*)P->J, (const R*)P->V0, (const R*)P->m,
                       (const R*)P->T, (const R*)P->gradT, (const R*)P->F);
  aux_join(c, s, c->ev_sjoin);
  // A1: parents, split masses, balance points, groups
  if (c->ns > 0)
    LAUNCH(c, MPM_K_SETUP, (k_parents<D, R>), dim3(cdiv(c->ns, 256 / kParGroup)), dim3(256), 0, s, d);
  if (c->np > 0) LAUNCH(c, MPM_K_SETUP, (k_split_mass<R>), dim3(cdiv(c->np, 256)), dim3(256), 0, s, d);
  scan(c, d.pcnt, d.grp_start, c->np, s);
  if (c->ns > 0) {
    LAUNCH(c, MPM_K_SETUP, (k_balance<D, R>), dim3(cdiv(c->ns, 256)), dim3(256), 0, s, d, c->sort_tmp);
    segment_order(c, (const int*)d.spar, (const int*)d.grp_start, c->ns, (const int*)c->sort_tmp, d.grp, s);
    cell_sort<D, R>(c, d, (const R*)d.bx_unsorted, c->ns, d.b_key, d.b_src, d.b_start, s, sort_res(c, d, false),
                    true);
    LAUNCH(c, MPM_K_SETUP, (k_gather_balance<D, R>), dim3(cdiv(c->ns, 256)), dim3(256), 0, s, d);
  }
  // active cell tiles (hold points) on this stream, node tiles on the second
  a = aux_fork(c, s, &c->ev_sfork);
  node_tiles<D, R>(c, d, a);
  aux_mark(c, a, &c->ev_sjoin);
  LAUNCH(c, MPM_K_SETUP, (k_flag_ctiles<D, R>), dim3(cdiv(c->ntile_total, 256)), dim3(256), 0, s, d, c->ctile_flag,
         c->ntile_total);
  scan(c, c->ctile_flag, c->ctile_pos, 2 * c->ntile_total, s);
  LAUNCH(c, MPM_K_SETUP, (k_ctile_slots<R>), dim3(cdiv(c->ntile_total, 256)), dim3(256), 0, s, d,
         (const int*)c->ctile_flag, (const int*)c->ctile_pos, c->ntile_total, c->ctile_list, c->ctile_slot,
         c->ctile_rng);
  HIPCHK(hipMemcpyAsync(c->hint + 1, c->ctile_pos + 2 * c->ntile_total, sizeof(int), hipMemcpyDeviceToHost, s));
  aux_join(c, s, c->ev_sjoin);
  host_mark(c, s, &c->ev_counts);
  // A2: the cell-tile scatter goes out before the host has the tile counts, sized by the
  // previous step's count (the kernel reads the true count); the host waits for the
  // counts while it runs and covers any further tiles with a second launch
  const int* nct_dev = c->ctile_pos + 2 * c->ntile_total;
  const int est = (int)std::min<int64_t>(c->ntile_total, c->prev_nctile + c->prev_nctile / 8 + 64);
  LAUNCH(c, MPM_K_P2G, (k_tile_p2g<D, R>), dim3(cdiv(est, 8) * 16), dim3(TileGeo<D>::NT), 0, s, d, tiles(c),
         (R*)c->tpart, nct_dev, 0);
  host_wait(c, s, c->ev_counts);
  c->ntiles = c->hint[0];
  c->nctile = c->hint[1];
  c->prev_ntiles = c->ntiles;
  c->prev_nctile = c->nctile;
  if (c->nctile > est)
    LAUNCH(c, MPM_K_P2G, (k_tile_p2g<D, R>), dim3(cdiv(c->nctile - est, 8) * 16), dim3(TileGeo<D>::NT), 0, s, d,
           tiles(c), (R*)c->tpart, nct_dev, est);
  // A2/A3: node merge of the scatter and grid set-up
  TileLists tl = tiles(c);
  if (c->ntiles > 0)
    LAUNCH(c, MPM_K_P2G_NODE, (k_merge_p2g<D, R>), dim3(c->ntiles), dim3(64), 0, s, d, tl, (const R*)c->tpart,
           c->nbr_slot);
  if (c->ns > 0) LAUNCH(c, MPM_K_SETUP, (k_surface_k<D, R>), dim3(cdiv(c->ns, 256)), dim3(256), 0, s, d);
  // degrees of freedom and whether any of them has a fixed component
  if (c->ntiles > 0)
    LAUNCH(c, MPM_K_SETUP, (k_dof_flags<D>), dim3(std::min(128, cdiv(c->ntiles, 4))), dim3(256), 0, s,
           (const int*)d.tile_list, c->ntiles * 64, (const uint8_t*)d.gfree, c->misc);
  c->have_p2g = true;
  const int64_t waits = c->stats.host_waits;   // counted since the step began
  c->stats = mpm_stats{};
  c->stats.host_waits = waits;
  c->stats.n_part = c->np;
  c->stats.n_surf = c->ns;
  c->stats.n_tiles = c->ntiles;
}


// Device scalar slots (doubles at ctx->scal).
// SC_G0 / SC_GT: the gradient merge's sums (see k_merge_stress) at the iterate and at the
// line-search trial: [0] Phi, [1..D] sum m (v^ - v^n), [D+1] sum m, [D+2] |g|^2, [D+3]
// the trial's slope g . delta, [D+4] the squared size of the gradient's terms (mixed_floor).
// SC_GO / SC_TOL2: the device's decision on the next Newton iteration (newton_decide).
enum : int { SC_DOT = 1, SC_RHS2 = 5, SC_MOM = 8, SC_G0 = 16, SC_GT = 32, SC_GO = 40, SC_TOL2 = 41, SC_N = 48 };
// MIXED Newton: the gradient is formed in FP32, so its norm cannot fall much below eps32
// times the size of the terms it is formed from (sums slot [D+4]).  Where the momentum is
// large against the forces this floor can sit above any fraction of |g0| worth asking for.
inline double mixed_floor(const double* sums, int D) {
  return 1.1920928955078125e-07 * std::sqrt(std::max(sums[D + 4], 0.0));
}
// The MIXED stop: |g| at its FP32 floor (below 1e-4 |g0|, or below mixed_floor) and the
// last Newton step did not halve it.
inline bool mixed_stop(double gn, double gn_prev, double g0, double fl) {
  return (gn <= 1e-4 * g0 || gn <= fl) && gn > 0.5 * gn_prev;
}
// MINRES scalars (momentum solve with krylov = MINRES) at scal[SC_N ..], inside the block
// the host reads back.
static_assert(SC_N * sizeof(double) + sizeof(MinresScal) <= (size_t)kScalDoubles * sizeof(double), "MINRES scalars");
inline MinresScal* minres_dev(mpm_ctx* c) { return (MinresScal*)(c->scal + SC_N); }
inline const MinresScal* minres_host(mpm_ctx* c) { return (const MinresScal*)(c->hbuf + SC_N); }

// Phi(u), the momentum sums and |g|^2 into scal[red_slot ..] (Phi also into energy_dev if
// given), projected gradient into g.
template <int D, typename R>
//
// With pu (z = v^, beta = alpha, p = the trial point) the point is v^ + alpha u, formed in
// the kernels and stored in pu.p; with slope_g the sums also hold slope_g . u; with fout
// the surface samples' F_r = I + dt grad v (the Hessian's linearization at this point).
void do_energy_grad(mpm_ctx* c, const R* u, R* g, double* energy_dev, int red_slot, hipStream_t s,
                    PUpd<R> pu = PUpd<R>{}, const R* slope_g = nullptr, R* fout = nullptr) {
  Dev<R>& d = dev<R>(c);
  TileLists tl = tiles(c);
  if (c->nctile > 0) {
    const int var = stress_var(d);
    if (var == SV_SOLID)
      LAUNCH(c, MPM_K_ENERGY_INT, (k_tile_stress<D, R, TM_ENERGY, SV_SOLID>), dim3(tile_grid(c)), dim3(TileGeo<D>::NT), sizeof(StressLds<D, R>),
             s, d, tl, u, (R*)c->tpart, 0, (const int*)nullptr, 2, pu, fout);
    else if (var == SV_JONLY)
      LAUNCH(c, MPM_K_ENERGY_INT, (k_tile_stress<D, R, TM_ENERGY, SV_JONLY>), dim3(tile_grid(c)), dim3(TileGeo<D>::NT), sizeof(StressLds<D, R>),
             s, d, tl, u, (R*)c->tpart, 0, (const int*)nullptr, 2, pu, fout);
    else
      LAUNCH(c, MPM_K_ENERGY_INT, (k_tile_stress<D, R, TM_ENERGY>), dim3(tile_grid(c)), dim3(TileGeo<D>::NT), sizeof(StressLds<D, R>), s, d,
             tl, u, (R*)c->tpart, 0, (const int*)nullptr, 2, pu, fout);
  }
  if (c->ntiles > 0) {
    LAUNCH(c, MPM_K_ENERGY_NODE, (k_merge_stress<D, R, NM_GRAD>), dim3(merge_blocks(c)), dim3(64 * kMergeTiles), 0, s, d, tl,
           c->ntiles, (const R*)c->tpart, u, g, 0.0, 0, (const int*)nullptr,
           c->nctile > 0 ? (const double*)(c->part + 2 * kPartSlot) : nullptr, c->nctile, c->part + 4 * kPartSlot,
           c->ctr + (size_t)CTR_MERGE * kCtrSite, c->scal + red_slot, energy_dev, (CgScal*)nullptr, pu, slope_g);
  } else {
    LAUNCH(c, MPM_K_BLAS, k_fill_r<double>, dim3(1), dim3(64), 0, s, c->scal + red_slot, 0.0, (int64_t)(D + 5));
    if (energy_dev) LAUNCH(c, MPM_K_BLAS, k_fill_r<double>, dim3(1), dim3(1), 0, s, energy_dev, 0.0, (int64_t)1);
  }
}

// Caches the surface linearization point F_r = I + dt grad v_lin(s_r).
template <int D, typename R>
void do_surface_lin(mpm_ctx* c, const R* vlin, hipStream_t s) {
  Dev<R>& d = dev<R>(c);
  if (c->ns > 0 && (d.term_mask & 2))
    LAUNCH(c, MPM_K_HESS_SURF, (k_surface_F<D, R>), dim3(cdiv(c->ns, 256)), dim3(256), 0, s, d, vlin);
  if (d.solids && c->np > 0)
    LAUNCH(c, MPM_K_HESS_SURF, (k_solid_lin<D, R>), dim3(cdiv(c->np, 256)), dim3(256), 0, s, d, vlin);
}

// out = P(alpha M P w + H P w) with the surface term linearized at the cached F_r.  With cg
// the merge also reduces w . out and sets the CG step length.  With z (a CG direction w):
// w is first replaced by z + beta w, which the merge stores.
// f_lin: the surface linearization to use instead of the cached one.
template <int D, typename R>
void do_hessvec(mpm_ctx* c, const R* w, double alpha, R* out, bool mask_in, const int* done, CgScal* cg,
                hipStream_t s, PUpd<R> pu = PUpd<R>{}, R* f_lin = nullptr) {
  Dev<R>& d = dev<R>(c);
  TileLists tl = tiles(c, TUNE_HESS);
  Dev<R> dh = d;
  if (f_lin) dh.sF = f_lin;
  if (c->nctile > 0) {
    const int var = stress_var(d);
    if (var == SV_SOLID)
      LAUNCH(c, MPM_K_HESS_INT, (k_tile_stress<D, R, TM_HESS, SV_SOLID>), dim3(tile_grid(c, TUNE_HESS)),
             dim3(TileGeo<D>::NT), sizeof(StressLds<D, R>), s, dh, tl, w, (R*)c->tpart, (int)mask_in, done, -1, pu, (R*)nullptr);
    else if (var == SV_JONLY)
      LAUNCH(c, MPM_K_HESS_INT, (k_tile_stress<D, R, TM_HESS, SV_JONLY>), dim3(tile_grid(c, TUNE_HESS)),
             dim3(TileGeo<D>::NT), sizeof(StressLds<D, R>), s, dh, tl, w, (R*)c->tpart, (int)mask_in, done, -1, pu, (R*)nullptr);
    else
      LAUNCH(c, MPM_K_HESS_INT, (k_tile_stress<D, R, TM_HESS>), dim3(tile_grid(c, TUNE_HESS)), dim3(TileGeo<D>::NT), sizeof(StressLds<D, R>),
             s, dh, tl, w, (R*)c->tpart, (int)mask_in, done, -1, pu, (R*)nullptr);
  }
  if (c->ntiles > 0)
    LAUNCH(c, MPM_K_HESS_NODE, (k_merge_stress<D, R, NM_HESS>), dim3(merge_blocks(c)), dim3(64 * kMergeTiles), 0, s, d, tl,
           c->ntiles, (const R*)c->tpart,
           w, out, alpha, (int)mask_in, done, (const double*)nullptr, 0, c->part + 4 * kPartSlot,
           c->ctr + (size_t)CTR_MERGE * kCtrSite, (double*)nullptr, (double*)nullptr, cg, pu, (const R*)nullptr);
}

// Forces only (no inertia term): out = P sum_q S_q grad N_i for the stress of u.
template <int D, typename R>
void do_hessvec_force(mpm_ctx* c, const R* u, R* out, hipStream_t s) {
  Dev<R>& d = dev<R>(c);
  TileLists tl = tiles(c);
  if (c->nctile > 0) {
    if (d.solids)
      LAUNCH(c, MPM_K_ENERGY_INT, (k_tile_stress<D, R, TM_FORCE, SV_SOLID>), dim3(tile_grid(c)), dim3(TileGeo<D>::NT), sizeof(StressLds<D, R>),
             s, d, tl, u, (R*)c->tpart, 0, (const int*)nullptr, -1, PUpd<R>{}, (R*)nullptr);
    else
      LAUNCH(c, MPM_K_ENERGY_INT, (k_tile_stress<D, R, TM_FORCE>), dim3(tile_grid(c)), dim3(TileGeo<D>::NT), sizeof(StressLds<D, R>), s, d,
             tl, u, (R*)c->tpart, 0, (const int*)nullptr, -1, PUpd<R>{}, (R*)nullptr);
  }
  if (c->ntiles > 0)
    LAUNCH(c, MPM_K_ENERGY_NODE, (k_merge_stress<D, R, NM_HESS>), dim3(merge_blocks(c)), dim3(64 * kMergeTiles), 0, s, d, tl,
           c->ntiles, (const R*)c->tpart,
           u, out, 0.0, 0, (const int*)nullptr, (const double*)nullptr, 0, c->part + 4 * kPartSlot,
           c->ctr + (size_t)CTR_MERGE * kCtrSite, (double*)nullptr, (double*)nullptr, (CgScal*)nullptr, PUpd<R>{},
           (const R*)nullptr);
}

// Uses only the heat solve's scratch (tile partials, partial slots 18.., counters CTR_H*),
// so that it can run beside the momentum solve.
template <int D, typename R>
void do_heat_apply(mpm_ctx* c, const R* T, R* out, const int* done, CgScal* cg, hipStream_t s,
                   PUpd<R> pu = PUpd<R>{}) {
  Dev<R>& d = dev<R>(c);
  TileLists tl = tiles(c, TUNE_HEAT);
  if (c->nctile > 0)
    LAUNCH(c, MPM_K_HEAT_PT, (k_tile_heat<D, R>), dim3(tile_grid(c, TUNE_HEAT)), dim3(TileGeo<D>::NT), 0, s, d, tl, T,
           (R*)c->tpart_heat, done, pu);
  if (c->ntiles > 0)
    LAUNCH(c, MPM_K_HEAT_NODE, (k_merge_heat<D, R>), dim3(merge_blocks(c)), dim3(64 * kMergeTiles), 0, s, d, tl,
           c->ntiles, (const R*)c->tpart_heat, T, out, done, c->part + 18 * kPartSlot,
           c->ctr + (size_t)CTR_HMERGE * kCtrSite, cg, pu);
}

template <int D, typename R>
void do_g2p(mpm_ctx* c, const R* vh, const R* Th, mpm_particles* P, hipStream_t s) {
  Dev<R>& d = dev<R>(c);
  if (!P || P->n != c->np) throw ApiError{MPM_EINVAL, "g2p particle count differs from p2g"};
  if (c->ns > 0) LAUNCH(c, MPM_K_G2P_SPLIT, (k_g2p_split<D, R>), dim3(cdiv(c->ns, 256)), dim3(256), 0, s, d, vh);
  if (c->nctile > 0)
    if (d.solids)
      LAUNCH(c, MPM_K_G2P, (k_tile_g2p<D, R, true>), dim3(c->nctile), dim3(256), 0, s, d, tiles(c), vh, Th,
             (R*)P->x, (R*)P->v, (R*)P->A, (R*)P->J, (R*)P->V0, (R*)P->m, (R*)P->T, (R*)P->gradT, (R*)P->F);
    else
      LAUNCH(c, MPM_K_G2P, (k_tile_g2p<D, R>), dim3(c->nctile), dim3(256), 0, s, d, tiles(c), vh, Th,
             (R*)P->x, (R*)P->v, (R*)P->A, (R*)P->J, (R*)P->V0, (R*)P->m, (R*)P->T, (R*)P->gradT, (R*)nullptr);
}

// a . b over the active nodes into scal[slot] (asynchronous).  heat: use the heat solve's
// partial slot and counter.
template <typename R>
void dot_async(mpm_ctx* c, const R* a, const R* b, int ncomp, int slot, hipStream_t s, bool heat = false) {
  Dev<R>& d = dev<R>(c);
  int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  LAUNCH(c, MPM_K_BLAS, k_dot<R>, dim3(nb), dim3(256), 0, s, (const int*)d.tile_list, nelem, d.nn, ncomp, a, b,
         c->part + (heat ? 19 * kPartSlot : 0), c->ctr + (size_t)(heat ? CTR_HDOT : CTR_DOT) * kCtrSite,
         c->scal + slot);
}

// Momentum sums of vh into scal[SC_MOM..] (asynchronous).
template <int D, typename R>
void mom_sums_async(mpm_ctx* c, const R* vh, hipStream_t s) {
  Dev<R>& d = dev<R>(c);
  int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  LAUNCH(c, MPM_K_BLAS, (k_mom_sums<D, R>), dim3(nb), dim3(kNodeThreads), 0, s, (const int*)d.tile_list, nelem, d.nn,
         (const uint8_t*)d.gfree, (const R*)d.gm, vh, (const R*)d.gvn, c->part, c->ctr + (size_t)CTR_MOM * kCtrSite, c->scal + SC_MOM);
}

// Reads the device scalar block (scalars, CG scalars, status words) in one copy and
// updates the latched status from it.
void read_mirror(mpm_ctx* c, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(c->hmirror, (const char*)c->scal, kMirrorRead, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c->stats.host_waits++;
  c->status |= c->hint[0];
  c->constrained = c->hint[1] != 0;
  c->stats.n_dof = c->hint[2];
}

// read_mirror in two halves, so that work can be queued behind the copy before the host
// waits for it.
void mirror_copy(mpm_ctx* c, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(c->hmirror, (const char*)c->scal, kMirrorRead, hipMemcpyDeviceToHost, s));
  host_mark(c, s, &c->ev_mread);
  c->mread_stream = s;
}
void mirror_wait(mpm_ctx* c) {
  host_wait(c, c->mread_stream, c->ev_mread);
  c->status |= c->hint[0];
  c->constrained = c->hint[1] != 0;
  c->stats.n_dof = c->hint[2];
}

// Jacobi-preconditioned CG with device-side scalars: apply(p, Ap, done, cg) must write
// A p and, when cg is given, set the step length from p . A p.  The kernels return at
// once after the done flag is set, so chunks of iterations can be queued ahead of the
// host's check: cg_begin queues the start and the first two iterations, cg_finish (after
// the host has read the scalars into hcg) queues further chunks of 4, 8, 16, ... until the
// flag is seen set, then the fix-up of a first-iteration breakdown.
struct CgRun {
  int chunk = 2;
  int launched = 0;
};

// Device scratch of one CG solve: its scalars (and their host mirror), partial slots and
// reduction counters.  Momentum and heat have separate sets.
// own_read: its host copy is a slot of its own, filled by kry_read (not by read_mirror).
struct KrySet {
  CgScal* cg;
  CgScal* hcg;
  double* part;
  unsigned* ctr_start;
  unsigned* ctr_upd;
  bool own_read;
};

// Momentum CG scalars: slot 0 for vector set 0, slot 2 for set 1 (slot 1 is the heat CG's).
inline KrySet kry_momentum(mpm_ctx* c, int set = 0) {
  return KrySet{c->cg + (set ? 2 : 0), c->hcg + (set ? 2 : 0), c->part, c->ctr + (size_t)CTR_CGSTART * kCtrSite,
                c->ctr + (size_t)CTR_CGUPD * kCtrSite, false};
}
inline KrySet kry_heat(mpm_ctx* c) {
  return KrySet{c->cg + 1, (CgScal*)(c->hmirror + kMirrorHeatHost), c->part + 16 * kPartSlot,
                c->ctr + (size_t)CTR_HSTART * kCtrSite, c->ctr + (size_t)CTR_HUPD * kCtrSite, true};
}

// Queues the copy of the solve's scalars to the host (with the whole mirror for the
// momentum solve); kry_read also waits for it.
void kry_copy(mpm_ctx* c, const KrySet& k, hipStream_t s) {
  if (k.own_read) HIPCHK(hipMemcpyAsync(k.hcg, k.cg, sizeof(CgScal), hipMemcpyDeviceToHost, s));
  else HIPCHK(hipMemcpyAsync(c->hmirror, (const char*)c->scal, kMirrorRead, hipMemcpyDeviceToHost, s));
}
void kry_read(mpm_ctx* c, const KrySet& k, hipStream_t s) {
  if (!k.own_read) {
    read_mirror(c, s);
    return;
  }
  kry_copy(c, k, s);
  HIPCHK(hipStreamSynchronize(s));
  c->stats.host_waits++;
}

// First chunk of a solve: the iteration count of the previous solve of the same kind
// (2..32).  Iterations queued past convergence return at once, while a chunk that is
// too short costs a host round trip, so the schedule follows the last count.
inline int first_chunk(int hint) { return std::max(2, std::min(hint, 32)); }

template <typename R, class Apply>
void cg_iterate(mpm_ctx* c, const KrySet& k, Apply&& apply, R* x, const R* diag, R* r, R* z, R* p, R* Ap, int ncomp,
                int n, hipStream_t s, CgRun& run) {
  Dev<R>& d = dev<R>(c);
  int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  const int* tl = d.tile_list;
  const int* done = &k.cg->done;
  // each operator application first forms the direction p = z + beta p (beta = 0 on the
  // first, which leaves p = z from the start)
  for (int j = 0; j < n; ++j) {
    apply(p, Ap, done, k.cg, PUpd<R>{p, z, k.cg});
    LAUNCH(c, MPM_K_BLAS, k_cg_update<R>, dim3(nb), dim3(kNodeThreads), 0, s, tl, nelem, d.nn, ncomp, k.cg, x, r, z,
           (const R*)p, (const R*)Ap, diag, k.part, k.ctr_upd);
  }
  run.launched += n;
}

template <typename R, class Apply>
void cg_begin(mpm_ctx* c, const KrySet& k, Apply&& apply, const R* b, double bscale, R* x, bool x0_given,
              const R* diag, R* r, R* z, R* p, R* Ap, int ncomp, double tol2_host, const double* tol2_scale, int maxit,
              hipStream_t s, CgRun& run, int first = 2, const double* gate = nullptr) {
  Dev<R>& d = dev<R>(c);
  int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  const int* tl = d.tile_list;
  if (x0_given) apply(x, Ap, (const int*)nullptr, (CgScal*)nullptr, PUpd<R>{});
  LAUNCH(c, MPM_K_BLAS, k_cg_start<R>, dim3(nb), dim3(kNodeThreads), 0, s, tl, nelem, d.nn, ncomp, b, (R)bscale,
         x0_given ? (const R*)Ap : (const R*)nullptr, diag, x, r, z, p, k.part, k.ctr_start, k.cg, tol2_host,
         tol2_scale, maxit, gate);
  run = CgRun{};
  run.chunk = std::min(first, std::max(maxit, 1));
  cg_iterate<R>(c, k, apply, x, diag, r, z, p, Ap, ncomp, run.chunk, s, run);
}

// Returns true when it changed x after the scalars in hcg were read (more iterations, or
// the breakdown fix-up), i.e. when work queued behind that read used an unfinished x.
template <typename R, class Apply>
bool cg_finish(mpm_ctx* c, const KrySet& k, Apply&& apply, R* x, const R* diag, R* r, R* z, R* p, R* Ap, int ncomp,
               int maxit, hipStream_t s, CgRun& run) {
  Dev<R>& d = dev<R>(c);
  int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  const int* tl = d.tile_list;
  bool changed = false;
  while (!k.hcg->done && run.launched < maxit + 32) {
    run.chunk = std::min(run.chunk * 2, 16);
    cg_iterate<R>(c, k, apply, x, diag, r, z, p, Ap, ncomp, run.chunk, s, run);
    kry_read(c, k, s);
    changed = true;
  }
  if (k.hcg->breakdown && k.hcg->iters == 0) {
    LAUNCH(c, MPM_K_BLAS, k_cg_fixup<R>, dim3(nb), dim3(256), 0, s, tl, nelem, d.nn, ncomp, (const CgScal*)k.cg, x,
           (const R*)z);
    changed = true;
  }
  if (!(k.hcg->rr == k.hcg->rr)) c->status |= ST_NONFINITE;
  return changed;
}

int status_code(int bits) {
  if (bits & (ST_STALL | ST_INTERNAL)) return MPM_EHIP;
  if (bits & ST_DOMAIN) return MPM_EDOMAIN;
  if (bits & ST_NONFINITE) return MPM_ENONFINITE;
  if (bits & ST_NOCONV) return MPM_ENOCONV;
  return MPM_OK;
}

// Status code of the latched status word (already read) with its message.
int status_code_of(mpm_ctx* c) {
  int code = status_code(c->status);
  if (code == MPM_EDOMAIN) c->err = "point outside [dx, 1-dx)^dim";
  else if (code == MPM_ENONFINITE) c->err = "non-finite residual or energy";
  else if (code == MPM_ENOCONV) c->err = "iteration cap reached";
  else if (code == MPM_EHIP) c->err = "a bounded device-side wait gave up or a device consistency check failed";
  return code;
}

template <int D, typename R>
void do_solve_momentum(mpm_ctx* c, hipStream_t s) {
  if (!c->have_p2g) throw ApiError{MPM_EINVAL, "mpm_p2g must run first"};
  Dev<R>& d = dev<R>(c);
  const mpm_params& p = c->p;
  int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  const int* tl = d.tile_list;
  R* vhat = (R*)c->vhat;
  R* vtrial = (R*)c->vtrial;
  R* g = (R*)c->grad;
  mpm_stats& st = c->stats;
  // start: v^ = P v^n; Phi, the mass sum and |g| come from the gradient merge.  The host
  // reads them together with the first iteration's CG and trial scalars: the first CG
  // chunk takes its tolerance from |g|^2 on the device, and the translation correction
  // tests the constrained flag on the device.  When the start already satisfies the
  // stopping test, that queued work is dropped (it writes only the CG and trial buffers).
  LAUNCH(c, MPM_K_BLAS, k_project_copy<R>, dim3(nb), dim3(256), 0, s, tl, nelem, d.nn, D, (const uint8_t*)d.gfree,
         (const R*)d.gvn, vhat);
  // the start's energy evaluation also caches the surface linearization F_r at v^; each
  // trial's goes to sF_alt, which becomes the cache when the trial is accepted
  do_energy_grad<D, R>(c, vhat, g, nullptr, SC_G0, s, PUpd<R>{}, nullptr, lin_cache(d) ? d.sF : nullptr);
  bool fix = false;
  double msum = 0, floor_abs = 0, phi = 0, gn = 0, g0 = 0, fl32 = 0;
  auto start_values = [&] {   // from a read that covers the start's gradient merge
    fix = p.momentum_fix && !c->constrained;
    msum = c->hbuf[SC_G0 + 1 + D];
    floor_abs = 1e-14 * msum * p.dx / p.dt;
    phi = c->hbuf[SC_G0];
    gn = std::sqrt(std::max(c->hbuf[SC_G0 + D + 2], 0.0));
    g0 = gn;
    fl32 = mixed_floor(c->hbuf + SC_G0, D);
    st.g0 = g0;
  };
  if (p.newton_max <= 0) {
    read_mirror(c, s);
    start_values();
  }
  st.energy_evals = 1;
  st.converged = 0;
  auto apply = [&](const R* pv, R* Apv, const int* done, CgScal* cg, PUpd<R> pu) {
    do_hessvec<D, R>(c, pv, 1.0, Apv, false, done, cg, s, pu);
  };
  const double eps = sizeof(R) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07;
  // CG vectors of the two sets (delta, r, z, p, Ap); iteration it uses set it % 2
  R* cgv[2][5] = {{(R*)c->delta, (R*)c->r, (R*)c->z, (R*)c->pp, (R*)c->Ap},
                  {(R*)c->cg2[0], (R*)c->cg2[1], (R*)c->cg2[2], (R*)c->cg2[3], (R*)c->cg2[4]}};
  int it = 0;
  double gn_prev = 1e300;
  bool have_next = false;   // this iteration's CG start and first chunk are already queued
  bool mom_formed = false;  // the momentum sums of v^ are in place (formed with its correction)
  CgRun next_run;
  for (; it < p.newton_max; ++it) {
    if (it > 0) {
      if (!(gn == gn) || !(phi == phi)) { c->status |= ST_NONFINITE; break; }
      if (gn <= std::max(p.newton_tol * g0, floor_abs)) { st.converged = 1; break; }
      // MIXED: the FP32 gradient cannot fall below its own round-off; once |g| is small
      // and a Newton step no longer halves it, the solve has reached that floor.
      if (sizeof(R) == 4 && mixed_stop(gn, gn_prev, g0, fl32)) { st.converged = 2; break; }
    }
    gn_prev = gn;
    const int set = it & 1;
    R* delta = cgv[set][0];
    R* cr = cgv[set][1];
    R* cz = cgv[set][2];
    R* cp = cgv[set][3];
    R* cAp = cgv[set][4];
    CgRun run;
    const KrySet km = kry_momentum(c, set);
    if (have_next) {
      // the queued start and first iteration, completed to the usual first chunk
      run = next_run;
      const int more = std::min(first_chunk(c->cg_hint_mom), std::max(p.cg_max, 1)) - run.launched;
      if (more > 0) {
        cg_iterate<R>(c, km, apply, delta, (const R*)d.gdiag, cr, cz, cp, cAp, D, more, s, run);
        run.chunk = run.launched;
      }
    } else if (it == 0) {
      // tolerance max(cg_rel |g|, 0.1 newton_tol |g0|) with g0 = |g|
      const double f = std::max(p.cg_rel, 0.1 * p.newton_tol);
      cg_begin<R>(c, km, apply, (const R*)g, -1.0, delta, false, (const R*)d.gdiag, cr, cz, cp, cAp, D, f * f,
                  c->scal + SC_G0 + D + 2, p.cg_max, s, run, first_chunk(c->cg_hint_mom));
    } else {
      const double cg_tol = std::max(p.cg_rel * gn, 0.1 * p.newton_tol * g0);
      cg_begin<R>(c, km, apply, (const R*)g, -1.0, delta, false, (const R*)d.gdiag, cr, cz, cp, cAp, D,
                  cg_tol * cg_tol, nullptr, p.cg_max, s, run, first_chunk(c->cg_hint_mom));
    }
    // the full step: the trial point v^ + alpha delta (formed in the energy kernels), its
    // energy and gradient with the slope g . delta, and the translation correction with
    // |g|^2 at the corrected point.  Queued behind the first CG chunk on the guess that
    // it converges there; the CG scalars and the trial's scalars come back in one read.
    // A trial that is rejected is overwritten by the next one, so the correction applied
    // speculatively is harmless.
    double alpha = 1.0;
    // The next iteration's CG start and first iteration (other vector set) are queued
    // behind the read, on the guess that the full step is accepted and the solve goes on:
    // the right side is the trial's gradient and the Hessian the trial's surface
    // linearization.  They keep the GPU busy while the host decides.  The device decides
    // with the host's tests whether they run (newton_decide); the host uses them only
    // when its own decision agrees and the trial stands as queued, else it starts the CG
    // afresh.  With the translation correction, the decision and the CG start are formed
    // by the correction's kernel.
    const bool spec = it + 1 < p.newton_max;
    R* const* nv = cgv[set ^ 1];
    const NewtonDecide nd{c->scal, D, (int)SC_GT, (int)SC_G0, it == 0 ? 1 : 0, phi, g0, floor_abs, gn, p.ls_c1,
                          8.0 * eps, p.ls_max > 1 ? 1 : 0, p.newton_tol, p.cg_rel, sizeof(R) == 4 ? 1 : 0,
                          p.dx / p.dt, (int)SC_GO, (int)SC_TOL2};
    auto trial_launch = [&](double a, bool first) {
      do_energy_grad<D, R>(c, (const R*)delta, (R*)c->gscratch, nullptr, SC_GT, s,
                           PUpd<R>{vtrial, (const R*)vhat, nullptr, (R)a}, (const R*)g,
                           lin_cache(d) ? (R*)c->sF_alt : nullptr);
      if (p.momentum_fix) {
        const bool fuse = first && spec;
        LAUNCH(c, MPM_K_BLAS, (k_mom_fix<D, R>), dim3(nb), dim3(kNodeThreads), 0, s, tl, nelem, d.nn, (const uint8_t*)d.gfree,
               (const R*)d.gm, (const double*)(c->scal + SC_GT + 1), p.dt, p.gravity[0], p.gravity[1], p.gravity[2],
               vtrial, (R*)c->gscratch, c->part, c->ctr + (size_t)CTR_MOM * kCtrSite, c->scal + SC_GT + D + 2,
               (const int*)(c->misc + 1), (const R*)d.gvn, c->scal + SC_MOM,
               fuse ? NextCgStart<R>{nv[0], nv[1], nv[2], nv[3], (const R*)d.gdiag, kry_momentum(c, set ^ 1).cg,
                                     p.cg_max}
                    : NextCgStart<R>{},
               fuse ? nd : NewtonDecide{});
      }
      st.energy_evals++;
    };
    trial_launch(alpha, true);
    if (spec && !p.momentum_fix)
      LAUNCH(c, MPM_K_BLAS, k_newton_decide, dim3(1), dim3(1), 0, s, nd, kry_momentum(c, set ^ 1).cg);
    mirror_copy(c, s);
    if (spec) {
      R* f_next = lin_cache(d) ? (R*)c->sF_alt : nullptr;
      auto apply_next = [&](const R* pv, R* Apv, const int* done, CgScal* cg, PUpd<R> pu) {
        do_hessvec<D, R>(c, pv, 1.0, Apv, false, done, cg, s, pu, f_next);
      };
      if (p.momentum_fix) {
        next_run = CgRun{};
        next_run.chunk = 1;
        cg_iterate<R>(c, kry_momentum(c, set ^ 1), apply_next, nv[0], (const R*)d.gdiag, nv[1], nv[2], nv[3], nv[4],
                      D, 1, s, next_run);
      } else {
        cg_begin<R>(c, kry_momentum(c, set ^ 1), apply_next, (const R*)c->gscratch, -1.0, nv[0], false,
                    (const R*)d.gdiag, nv[1], nv[2], nv[3], nv[4], D, 1.0, c->scal + SC_TOL2, p.cg_max, s, next_run,
                    1, c->scal + SC_GO);
      }
    }
    mirror_wait(c);
    const bool dev_go = c->hbuf[SC_GO] != 0.0;
    have_next = false;
    if (it == 0) {
      start_values();
      if (!(gn == gn) || !(phi == phi)) { c->status |= ST_NONFINITE; st.energy_evals--; break; }
      if (gn <= std::max(p.newton_tol * g0, floor_abs)) { st.converged = 1; st.energy_evals--; break; }
    }
    bool stands = true;   // the trial read above is the one accepted, at alpha = 1
    if (cg_finish<R>(c, km, apply, delta, (const R*)d.gdiag, cr, cz, cp, cAp, D, p.cg_max, s, run)) {
      // the guess failed: the trial used an unfinished delta
      trial_launch(alpha, false);
      read_mirror(c, s);
      stands = false;
    }
    const int cit = km.hcg->iters;
    c->cg_hint_mom = cit;
    st.cg_iters += cit;
    st.hessvecs += cit;
    const double slope = c->hbuf[SC_GT + D + 3];
    double phit = c->hbuf[SC_GT];
    // Armijo with the round-off of Phi as allowance (8 eps |Phi|, eps of the arithmetic):
    // near convergence the decrement is below it and the test would be decided by noise.
    for (int ls = 1; ls < std::max(p.ls_max, 1); ++ls) {
      const double noise = 8.0 * eps * std::max(std::fabs(phi), std::fabs(phit));
      if (phit <= phi + p.ls_c1 * alpha * slope + noise) break;
      alpha *= 0.5;
      st.line_search_halvings++;
      trial_launch(alpha, false);
      read_mirror(c, s);
      phit = c->hbuf[SC_GT];
      stands = false;
    }
    have_next = spec && dev_go && stands;
    // accept the last trial: its (corrected) point and gradient become the iterate; its
    // momentum sums, when the correction's kernel formed them, are the solve's
    mom_formed = p.momentum_fix;
    std::swap(c->vhat, c->vtrial);
    {
      R* f_acc = (R*)c->sF_alt;
      c->sF_alt = d.sF;
      d.sF = f_acc;
    }
    std::swap(c->grad, c->gscratch);
    vhat = (R*)c->vhat;
    vtrial = (R*)c->vtrial;
    g = (R*)c->grad;
    phi = phit;
    if (fix) {
      // Phi(v^ - c) = Phi(v^) - 1/2 |c|^2 sum m for the minimizing translation c
      const double* red = c->hbuf + SC_GT + 1;
      const double M = red[D];
      double c2 = 0;
      for (int a2 = 0; a2 < D; ++a2) {
        double ca = (red[a2] - p.dt * p.gravity[a2] * M) / M;
        c2 += ca * ca;
      }
      phi -= 0.5 * M * c2;
    }
    gn = std::sqrt(std::max(c->hbuf[SC_GT + D + 2], 0.0));
    fl32 = mixed_floor(c->hbuf + SC_GT, D);
  }
  if (it == p.newton_max && gn <= std::max(p.newton_tol * g0, floor_abs)) st.converged = 1;
  st.newton_iters = it;
  st.gnorm = gn;
  st.phi = phi;
  if (!st.converged && !(c->status & ST_NONFINITE)) c->status |= ST_NOCONV;
  // grid momentum after the solve (read with the next status query)
  if (!mom_formed) mom_sums_async<D, R>(c, (const R*)vhat, s);
  c->mom_pending = true;
}

// Preconditioned MINRES on the projected Newton system for the right side bscale * b,
// into x; stops at phibar <= rel_tol phibar_0 or after maxit iterations.  Uses the two CG
// vector sets (nine vectors) and the CG reduction slots.  Chunks of iterations are queued
// ahead of the host's check, as for CG; iterations past convergence return at once.
// Returns the iteration count.
template <int D, typename R>
int minres_solve(mpm_ctx* c, const R* b, double bscale, R* x, double rel_tol, int maxit, hipStream_t s) {
  Dev<R>& d = dev<R>(c);
  const int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  const int* tl = d.tile_list;
  MinresScal* ms = minres_dev(c);
  R* y = (R*)c->r;
  R* t = (R*)c->z;
  R* v = (R*)c->pp;
  R* rp = (R*)c->Ap;
  R* rc = (R*)c->cg2[0];
  R* w = (R*)c->cg2[1];
  R* wp = (R*)c->cg2[2];
  unsigned* ctr_a = c->ctr + (size_t)CTR_CGSTART * kCtrSite;
  unsigned* ctr_b = c->ctr + (size_t)CTR_CGUPD * kCtrSite;
  LAUNCH(c, MPM_K_BLAS, k_minres_start<R>, dim3(nb), dim3(kNodeThreads), 0, s, tl, nelem, d.nn, D, b, (R)bscale,
         (const R*)d.gdiag, x, rp, rc, y, w, wp, c->part, ctr_a, ms, rel_tol, maxit);
  int launched = 0, chunk = first_chunk(c->cg_hint_mom);
  for (;;) {
    for (int j = 0; j < chunk; ++j) {
      do_hessvec<D, R>(c, (const R*)y, 1.0, t, false, &ms->done, (CgScal*)nullptr, s);
      LAUNCH(c, MPM_K_BLAS, k_minres_lanczos<R>, dim3(nb), dim3(kNodeThreads), 0, s, tl, nelem, d.nn, D, (const R*)y,
             t, v, (const R*)rp, c->part, ctr_a, ms);
      LAUNCH(c, MPM_K_BLAS, k_minres_rotate<R>, dim3(nb), dim3(kNodeThreads), 0, s, tl, nelem, d.nn, D, t,
             (const R*)rc, (const R*)d.gdiag, y, c->part, ctr_b, ms);
      LAUNCH(c, MPM_K_BLAS, k_minres_step<R>, dim3(nb), dim3(kNodeThreads), 0, s, tl, nelem, d.nn, D, (const R*)v,
             (const R*)w, wp, x, (const MinresScal*)ms, launched + j + 1);
      // (r_prev, r_cur) <- (r_cur, t); t takes the old r_prev; (w_prev, w) <- (w, w')
      R* old_rp = rp;
      rp = rc;
      rc = t;
      t = old_rp;
      std::swap(w, wp);
    }
    launched += chunk;
    read_mirror(c, s);
    if (minres_host(c)->done || launched >= maxit + 32) break;
    chunk = std::min(chunk * 2, 16);
  }
  const MinresScal* hm = minres_host(c);
  if (hm->breakdown) c->status |= ST_NONFINITE;
  c->cg_hint_mom = hm->iters;
  return hm->iters;
}

// Newton on Phi with each step solved by MINRES (krylov = MINRES), in the order of the
// oracle's Newton loop: no work is queued ahead of the host's decisions.  Same stopping
// tests, Armijo line search and translation correction as the CG path.
template <int D, typename R>
void do_solve_momentum_minres(mpm_ctx* c, hipStream_t s) {
  if (!c->have_p2g) throw ApiError{MPM_EINVAL, "mpm_p2g must run first"};
  Dev<R>& d = dev<R>(c);
  const mpm_params& p = c->p;
  const int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  const int* tl = d.tile_list;
  mpm_stats& st = c->stats;
  LAUNCH(c, MPM_K_BLAS, k_project_copy<R>, dim3(nb), dim3(256), 0, s, tl, nelem, d.nn, D, (const uint8_t*)d.gfree,
         (const R*)d.gvn, (R*)c->vhat);
  do_energy_grad<D, R>(c, (const R*)c->vhat, (R*)c->grad, nullptr, SC_G0, s, PUpd<R>{}, nullptr,
                       lin_cache(d) ? d.sF : nullptr);
  read_mirror(c, s);
  const bool fix = p.momentum_fix && !c->constrained;
  const double msum = c->hbuf[SC_G0 + 1 + D];
  const double floor_abs = 1e-14 * msum * p.dx / p.dt;
  double phi = c->hbuf[SC_G0];
  double gn = std::sqrt(std::max(c->hbuf[SC_G0 + D + 2], 0.0));
  const double g0 = gn;
  double fl32 = mixed_floor(c->hbuf + SC_G0, D);
  st.g0 = g0;
  st.energy_evals = 1;
  st.converged = 0;
  const double eps = sizeof(R) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07;
  int it = 0;
  double gn_prev = 1e300;
  for (; it < p.newton_max; ++it) {
    if (!(gn == gn) || !(phi == phi)) { c->status |= ST_NONFINITE; break; }
    if (gn <= std::max(p.newton_tol * g0, floor_abs)) { st.converged = 1; break; }
    // MIXED: the FP32 gradient's round-off floor, as in the CG path
    if (sizeof(R) == 4 && it > 0 && mixed_stop(gn, gn_prev, g0, fl32)) { st.converged = 2; break; }
    gn_prev = gn;
    const double cg_tol = std::max(p.cg_rel * gn, 0.1 * p.newton_tol * g0);
    R* delta = (R*)c->delta;
    const int kit = minres_solve<D, R>(c, (const R*)c->grad, -1.0, delta, cg_tol / gn, p.cg_max, s);
    st.cg_iters += kit;
    st.hessvecs += kit;
    auto trial = [&](double a) {
      do_energy_grad<D, R>(c, (const R*)delta, (R*)c->gscratch, nullptr, SC_GT, s,
                           PUpd<R>{(R*)c->vtrial, (const R*)c->vhat, nullptr, (R)a}, (const R*)c->grad,
                           lin_cache(d) ? (R*)c->sF_alt : nullptr);
      if (p.momentum_fix)
        LAUNCH(c, MPM_K_BLAS, (k_mom_fix<D, R>), dim3(nb), dim3(kNodeThreads), 0, s, tl, nelem, d.nn,
               (const uint8_t*)d.gfree, (const R*)d.gm, (const double*)(c->scal + SC_GT + 1), p.dt, p.gravity[0],
               p.gravity[1], p.gravity[2], (R*)c->vtrial, (R*)c->gscratch, c->part,
               c->ctr + (size_t)CTR_MOM * kCtrSite, c->scal + SC_GT + D + 2, (const int*)(c->misc + 1),
               (const R*)d.gvn, c->scal + SC_MOM, NextCgStart<R>{}, NewtonDecide{});
      st.energy_evals++;
      read_mirror(c, s);
    };
    double alpha = 1.0;
    trial(alpha);
    const double slope = c->hbuf[SC_GT + D + 3];
    double phit = c->hbuf[SC_GT];
    for (int ls = 1; ls < std::max(p.ls_max, 1); ++ls) {
      const double noise = 8.0 * eps * std::max(std::fabs(phi), std::fabs(phit));
      if (phit <= phi + p.ls_c1 * alpha * slope + noise) break;
      alpha *= 0.5;
      st.line_search_halvings++;
      trial(alpha);
      phit = c->hbuf[SC_GT];
    }
    // accept the last trial (its corrected point, gradient and surface linearization)
    std::swap(c->vhat, c->vtrial);
    {
      R* f_acc = (R*)c->sF_alt;
      c->sF_alt = d.sF;
      d.sF = f_acc;
    }
    std::swap(c->grad, c->gscratch);
    phi = phit;
    if (fix) {
      const double* red = c->hbuf + SC_GT + 1;
      const double M = red[D];
      double c2 = 0;
      for (int a2 = 0; a2 < D; ++a2) {
        const double ca = (red[a2] - p.dt * p.gravity[a2] * M) / M;
        c2 += ca * ca;
      }
      phi -= 0.5 * M * c2;
    }
    gn = std::sqrt(std::max(c->hbuf[SC_GT + D + 2], 0.0));
    fl32 = mixed_floor(c->hbuf + SC_GT, D);
  }
  if (it == p.newton_max && gn <= std::max(p.newton_tol * g0, floor_abs)) st.converged = 1;
  st.newton_iters = it;
  st.gnorm = gn;
  st.phi = phi;
  if (!st.converged && !(c->status & ST_NONFINITE)) c->status |= ST_NOCONV;
  if (p.momentum_fix && it > 0) {
    // the momentum sums of the accepted point were formed by its translation correction
  } else {
    mom_sums_async<D, R>(c, (const R*)c->vhat, s);
  }
  c->mom_pending = true;
}

template <int D, typename R>
void do_explicit(mpm_ctx* c, hipStream_t s) {
  if (!c->have_p2g) throw ApiError{MPM_EINVAL, "mpm_p2g must run first"};
  Dev<R>& d = dev<R>(c);
  int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  const int* tl = d.tile_list;
  R* f = (R*)c->grad;
  R* f2 = (R*)c->gscratch;
  R* zero = (R*)c->zero;
  LAUNCH(c, MPM_K_BLAS, k_axpy_to<R>, dim3(nb), dim3(256), 0, s, tl, nelem, d.nn, D, (const R*)d.gvn, (const R*)d.gvn,
         -1.0, zero);
  Dev<R> saved = d;
  // J and surface terms at y = x (v^ = 0)
  d.term_mask = saved.term_mask & 3;
  do_hessvec_force<D, R>(c, zero, f, s);
  // viscous term at the strain rate of v^n
  d.term_mask = saved.term_mask & 4;
  if (d.term_mask) {
    do_hessvec_force<D, R>(c, (const R*)d.gvn, f2, s);
    LAUNCH(c, MPM_K_BLAS, k_axpy_to<R>, dim3(nb), dim3(256), 0, s, tl, nelem, d.nn, D, (const R*)f, (const R*)f2, 1.0,
           f);
  }
  d = saved;
  LAUNCH(c, MPM_K_BLAS, (k_explicit_update<D, R>), dim3(nb), dim3(256), 0, s, tl, nelem, d.nn, (const uint8_t*)d.gfree,
         (const R*)d.gm, (const R*)d.gvn, (const R*)f, (R)c->p.gravity[0], (R)c->p.gravity[1], (R)c->p.gravity[2],
         (R)c->p.dt, (R*)c->vhat);
  c->stats.converged = 1;
  mom_sums_async<D, R>(c, (const R*)c->vhat, s);
  c->mom_pending = true;
}

// Heat solve, split so that work can be queued behind its first CG chunk: heat_begin
// queues T = T^n, |rhs|^2, the CG start with its first iterations and the copy of the CG
// scalars to their host slot; heat_end waits for that copy, finishes the CG and records
// the statistics, returning true when it changed T^ after the copy.  The heat solve uses
// only its own scratch (kry_heat, its tile partials, its host slot), so it may run on a
// second stream beside the momentum solve.
template <int D, typename R>
void heat_begin(mpm_ctx* c, hipStream_t s, CgRun& run) {
  if (!c->have_p2g) throw ApiError{MPM_EINVAL, "mpm_p2g must run first"};
  Dev<R>& d = dev<R>(c);
  int nelem = c->ntiles * 64, nb = krylov_blocks(nelem);
  const int* tl = d.tile_list;
  R* T = (R*)c->That;
  LAUNCH(c, MPM_K_BLAS, k_axpy_to<R>, dim3(nb), dim3(256), 0, s, tl, nelem, d.nn, 1, (const R*)d.gTn, (const R*)d.gTn,
         0.0, T);
  dot_async<R>(c, (const R*)d.hrhs, (const R*)d.hrhs, 1, SC_RHS2, s, true);
  auto apply = [&](const R* pv, R* Apv, const int* done, CgScal* cg, PUpd<R> pu) {
    do_heat_apply<D, R>(c, pv, Apv, done, cg, s, pu);
  };
  const KrySet kh = kry_heat(c);
  cg_begin<R>(c, kh, apply, d.hrhs, 1.0, T, true, (const R*)d.hdiag, (R*)c->hr, (R*)c->hz, (R*)c->hp,
              (R*)c->hAp, 1, c->p.heat_tol * c->p.heat_tol, c->scal + SC_RHS2, c->p.heat_max, s, run,
              first_chunk(c->cg_hint_heat));
  // the scalars after the first chunk go to the host at once; heat_end waits for them
  kry_copy(c, kh, s);
  host_mark(c, s, &c->ev_hread);
}

template <int D, typename R>
bool heat_end(mpm_ctx* c, hipStream_t s, CgRun& run) {
  Dev<R>& d = dev<R>(c);
  const KrySet kh = kry_heat(c);
  host_wait(c, s, c->ev_hread);
  auto apply = [&](const R* pv, R* Apv, const int* done, CgScal* cg, PUpd<R> pu) {
    do_heat_apply<D, R>(c, pv, Apv, done, cg, s, pu);
  };
  bool changed = cg_finish<R>(c, kh, apply, (R*)c->That, (const R*)d.hdiag, (R*)c->hr, (R*)c->hz, (R*)c->hp,
                              (R*)c->hAp, 1, c->p.heat_max, s, run);
  const int it = kh.hcg->iters;
  c->cg_hint_heat = it;
  c->stats.heat_iters = it;
  c->stats.heat_res = std::sqrt(std::max(kh.hcg->rr, 0.0));
  if (it >= c->p.heat_max && kh.hcg->rr > kh.hcg->tol2) c->status |= ST_NOCONV;
  return changed;
}

template <int D, typename R>
void do_solve_heat(mpm_ctx* c, hipStream_t s) {
  CgRun run;
  heat_begin<D, R>(c, s, run);
  heat_end<D, R>(c, s, run);
}

// Device surface sampler (Section 4.1.1; kernels in sampler_dev.h).  Returns the sample
// count; the samples are written only when it is <= cap.
template <int D, typename R>
int64_t do_sample(mpm_ctx* c, const mpm_particles* P, const SmpArgs& a, R* s_out, R* dA_out, int* label,
                  int64_t cap, hipStream_t s) {
  Dev<R>& d = dev<R>(c);
  const int np = (int)P->n;
  if (np <= 0) return 0;
  const int n = a.n;
  const int64_t nn = c->nn;
  const int64_t ncube = (int64_t)(n - 1) * (n - 1) * (D == 3 ? (n - 1) : 1);
  const R* x = (const R*)P->x;
  // binning: keys and counts, dense cell starts, slots, each cell's segment in input order
  LAUNCH(c, MPM_K_SAMPLE, (k_smp_keys<D, R>), dim3(cdiv(np, 256)), dim3(256), 0, s, x, np, n, c->nt, a.dx,
         c->smp_key, d.ccount);
  scan(c, d.ccount, c->smp_start, (int)nn, s);
  LAUNCH(c, MPM_K_SAMPLE, k_cell_scatter, dim3(cdiv(np, 256)), dim3(256), 0, s, (const int*)c->smp_key, np,
         (const int*)c->smp_start, d.ccount, c->sort_tmp, d.status);
  segment_order(c, c->smp_key, c->smp_start, np, (const int*)c->sort_tmp, c->smp_perm, s);
  LAUNCH(c, MPM_K_SAMPLE, (k_smp_gather<D, R>), dim3(cdiv(np, 256)), dim3(256), 0, s, x, np,
         (const int*)c->smp_perm, d.px);
  // the level set near the particles
  LAUNCH(c, MPM_K_SAMPLE, k_fill_i32, dim3(cdiv(nn / 4, 256)), dim3(256), 0, s, (int*)c->smp_flag, 0,
         (int64_t)(nn / 4));
  LAUNCH(c, MPM_K_SAMPLE, (k_smp_inside<D, R>), dim3(cdiv(np, 256)), dim3(256), 0, s, x, np, a, c->smp_flag);
  LAUNCH(c, MPM_K_SAMPLE, (k_smp_need<D>), dim3(cdiv(nn, 256)), dim3(256), 0, s, c->smp_flag, n);
  LAUNCH(c, MPM_K_SAMPLE, (k_smp_phi<D, R>), dim3(cdiv(nn, 256)), dim3(256), 0, s, (const R*)d.px, np,
         (const int*)c->smp_start, a, (const uint8_t*)c->smp_flag, c->smp_phi);
  // elements and samples, in element-id order
  LAUNCH(c, MPM_K_SAMPLE, (k_smp_count<D>), dim3(cdiv(ncube, 256)), dim3(256), 0, s, a,
         (const uint8_t*)c->smp_flag, (const double*)c->smp_phi, c->smp_cnt);
  scan(c, c->smp_cnt, c->smp_off, (int)ncube, s);
  LAUNCH(c, MPM_K_SAMPLE, (k_smp_emit<D, R>), dim3(cdiv(ncube, 256)), dim3(256), 0, s, a,
         (const uint8_t*)c->smp_flag, (const double*)c->smp_phi, (const int*)c->smp_cnt, (const int*)c->smp_off,
         cap, s_out, dA_out, label);
  HIPCHK(hipGetLastError());
  int total = 0;
  sync_read(c, s, c->smp_off + ncube, &total, sizeof(int));
  return total;
}

// ---- dispatch ----------------------------------------------------------------------------
template <class F>
void dispatch(mpm_ctx* c, F&& f) {
  if (c->dim == 3) {
    if (c->fp64) f(std::integral_constant<int, 3>{}, double{});
    else f(std::integral_constant<int, 3>{}, float{});
  } else {
    if (c->fp64) f(std::integral_constant<int, 2>{}, double{});
    else f(std::integral_constant<int, 2>{}, float{});
  }
}

// Message of the last failure that had no context to hold it (mpm_last_error(NULL)).
thread_local std::string g_last_error;

template <class F>
int guarded(mpm_ctx* c, F&& f) {
  std::string& err = c ? c->err : g_last_error;
  try {
    f();
    return MPM_OK;
  } catch (const ApiError& e) {
    err = e.msg;
    return e.code;
  } catch (const HipError& e) {
    err = std::string(e.what) + ": " + hipGetErrorString(e.e);
    return MPM_EHIP;
  } catch (...) {
    err = "unexpected exception";
    return MPM_EHIP;
  }
}

int check_launch(mpm_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    c->err = std::string("kernel launch: ") + hipGetErrorString(e);
    return MPM_EHIP;
  }
  return MPM_OK;
}

// Workspace bytes of a context with parameters p and the given capacities.
size_t workspace_need(const mpm_params* p, int64_t cap_part, int64_t cap_surf) {
  check_params(p);
  if (cap_part < 0 || cap_surf < 0) throw ApiError{MPM_EINVAL, "bad arguments"};
  if (cap_part > (int64_t)kScanBlock * kScanBlock || cap_surf > (int64_t)kScanBlock * kScanBlock)
    throw ApiError{MPM_EINVAL, "capacity above 2^24"};
  mpm_ctx tmp;
  tmp.p = *p;
  tmp.dim = p->dim;
  tmp.n = p->n;
  tmp.nn = 1;
  for (int a = 0; a < p->dim; ++a) tmp.nn *= p->n;
  tmp.ntile_total = tmp.nn / 64;
  tmp.cap_part = cap_part;
  tmp.cap_surf = cap_surf;
  return p->precision == MPM_FP64 ? layout<double>(&tmp, nullptr) : layout<float>(&tmp, nullptr);
}

// Sets up context c over the device workspace ws (need bytes are used) and the host
// mirror block (kMirrorBytes): the parameters, the workspace carving and the per-step
// state, and zeroes the used workspace with a fill kernel on stream s (the cell counters
// and scan status words must start at zero), waiting for it.  Allocates nothing.
void ctx_init(mpm_ctx* c, const mpm_params* p, void* ws, size_t ws_bytes, size_t need, int64_t cap_part,
              int64_t cap_surf, char* mirror, hipStream_t s) {
  c->p = *p;
  c->dim = p->dim;
  c->n = p->n;
  c->nt = p->n / (p->dim == 3 ? 4 : 8);
  c->nn = 1;
  for (int a = 0; a < p->dim; ++a) c->nn *= p->n;
  c->ntile_total = c->nn / 64;
  c->cap_part = cap_part;
  c->cap_surf = cap_surf;
  c->fp64 = p->precision == MPM_FP64;
  c->ws = (char*)ws;
  c->ws_bytes = ws_bytes;
  c->d64 = Dev<double>{};
  c->d32 = Dev<float>{};
  if (c->fp64) {
    layout<double>(c, c->ws);
    fill_params(c->d64, *p, c->nt);
  } else {
    layout<float>(c, c->ws);
    fill_params(c->d32, *p, c->nt);
  }
  c->hmirror = mirror;
  c->hbuf = (double*)c->hmirror;
  c->hcg = (CgScal*)(c->hmirror + kMirrorCg);
  c->hint = (int*)(c->hmirror + kMirrorMisc);
  c->nctile = 0;
  c->scan_epoch = c->scan_epoch_aux = 0;
  c->np = c->ns = c->ntiles = c->prev_ntiles = c->prev_nctile = 0;
  c->have_p2g = c->constrained = c->mom_pending = false;
  c->cg_hint_mom = c->cg_hint_heat = 2;
  c->status = 0;
  c->stats = mpm_stats{};
  c->err.clear();
  HIPCHK(hipGetDevice(&c->device));
  hipLaunchKernelGGL(k_fill_i32, dim3(cdiv((int64_t)(need / 4), 256)), dim3(256), 0, s, (int*)c->ws, 0,
                     (int64_t)(need / 4));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
}

}  // namespace

// =========================================================================================
// C ABI
// =========================================================================================
extern "C" {

int mpm_params_default(mpm_params* p, int32_t dim, int32_t n) {
  if (!p || (dim != 2 && dim != 3) || n <= 0) return MPM_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->dim = dim;
  p->n = n;
  p->dx = 1.0 / n;
  p->dt = 1e-3;
  p->precision = MPM_FP64;
  p->hess_mode = MPM_HESS_PSD;
  p->term_mask = 7;
  p->momentum_fix = 1;
  p->slab_axis = 1;
  p->newton_max = 20;
  p->cg_max = 1000;
  p->ls_max = 10;
  p->heat_max = 1000;
  p->bulk = 1e4;
  p->gmax = 1e30;
  p->cp = 1.0;
  p->newton_tol = 1e-8;
  p->cg_rel = 1e-2;
  p->ls_c1 = 1e-4;
  p->heat_tol = 1e-10;
  return MPM_OK;
}

int mpm_workspace_bytes(const mpm_params* p, int64_t cap_part, int64_t cap_surf, size_t* out_bytes) {
  return guarded(nullptr, [&] {
    if (!out_bytes) throw ApiError{MPM_EINVAL, "bad arguments"};
    *out_bytes = workspace_need(p, cap_part, cap_surf);
  });
}

int mpm_ctx_create(const mpm_params* p, void* workspace, size_t ws_bytes, int64_t cap_part, int64_t cap_surf,
                   mpm_ctx** out) {
  if (!out) return MPM_EINVAL;
  *out = nullptr;
  size_t need = 0;
  int rc = mpm_workspace_bytes(p, cap_part, cap_surf, &need);
  if (rc != MPM_OK) return rc;
  if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255)) return MPM_EINVAL;
  mpm_ctx* c = new mpm_ctx();
  rc = guarded(c, [&] {
    HIPCHK(hipHostMalloc((void**)&c->hmirror, kMirrorBytes, hipHostMallocDefault));
    ctx_init(c, p, workspace, ws_bytes, need, cap_part, cap_surf, c->hmirror, nullptr);
  });
  if (rc != MPM_OK) {
    g_last_error = c->err;
    if (c->hmirror) hipHostFree(c->hmirror);
    delete c;
    return rc;
  }
  *out = c;
  return MPM_OK;
}

int mpm_ctx_destroy(mpm_ctx* ctx) {
  if (!ctx) return MPM_EINVAL;
  for (hipEvent_t e : ctx->prof.ev) hipEventDestroy(e);
  if (ctx->own) {
    hipStreamSynchronize(ctx->own);
    hipStreamDestroy(ctx->own);
  }
  if (ctx->own_done) hipEventDestroy(ctx->own_done);
  if (ctx->aux) {
    hipStreamSynchronize(ctx->aux);
    hipStreamDestroy(ctx->aux);
  }
  if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
  if (ctx->ev_hread) hipEventDestroy(ctx->ev_hread);
  if (ctx->ev_counts) hipEventDestroy(ctx->ev_counts);
  if (ctx->ev_sfork) hipEventDestroy(ctx->ev_sfork);
  if (ctx->ev_sjoin) hipEventDestroy(ctx->ev_sjoin);
  if (ctx->ev_mread) hipEventDestroy(ctx->ev_mread);
  if (ctx->hmirror) hipHostFree(ctx->hmirror);
  delete ctx;
  return MPM_OK;
}

const char* mpm_last_error(const mpm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

int mpm_ctx_set_params(mpm_ctx* ctx, const mpm_params* p) {
  if (!ctx) return MPM_EINVAL;
  return guarded(ctx, [&] {
    check_params(p);
    if (p->dim != ctx->dim || p->n != ctx->n || (p->precision == MPM_FP64) != ctx->fp64)
      throw ApiError{MPM_EINVAL, "dim, n and precision are fixed per context"};
    if (solids_on(*p) && !(ctx->fp64 ? ctx->d64.solids : ctx->d32.solids))
      throw ApiError{MPM_EINVAL, "solids (T_melt) need a context created with them"};
    ctx->p = *p;
    if (ctx->fp64) fill_params(ctx->d64, *p, ctx->nt);
    else fill_params(ctx->d32, *p, ctx->nt);
  });
}

int mpm_p2g(mpm_ctx* ctx, const mpm_particles* P, const mpm_surface* S, void* stream) {
  if (!ctx) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(ctx, [&] {
    ctx->status = 0;
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      do_p2g<D, R>(ctx, P, S, s);
    });
  });
  return rc != MPM_OK ? rc : check_launch(ctx);
}

int mpm_energy_grad(mpm_ctx* ctx, const void* v_hat, double* energy_dev, void* grad, void* stream) {
  if (!ctx || !v_hat || !grad) return MPM_EINVAL;
  if (!ctx->have_p2g) { ctx->err = "mpm_p2g must run first"; return MPM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(ctx, [&] {
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      do_energy_grad<D, R>(ctx, (const R*)v_hat, (R*)grad, energy_dev, SC_G0, s);
    });
  });
  return rc != MPM_OK ? rc : check_launch(ctx);
}

int mpm_hessvec(mpm_ctx* ctx, const void* v_lin, const void* w, double alpha_mass, void* out, void* stream) {
  if (!ctx || !v_lin || !w || !out) return MPM_EINVAL;
  if (!ctx->have_p2g) { ctx->err = "mpm_p2g must run first"; return MPM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(ctx, [&] {
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      do_surface_lin<D, R>(ctx, (const R*)v_lin, s);
      do_hessvec<D, R>(ctx, (const R*)w, alpha_mass, (R*)out, true, nullptr, (CgScal*)nullptr, s);
    });
  });
  return rc != MPM_OK ? rc : check_launch(ctx);
}

int mpm_heat_apply(mpm_ctx* ctx, const void* T_in, void* T_out, void* stream) {
  if (!ctx || !T_in || !T_out) return MPM_EINVAL;
  if (!ctx->have_p2g) { ctx->err = "mpm_p2g must run first"; return MPM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(ctx, [&] {
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      do_heat_apply<D, R>(ctx, (const R*)T_in, (R*)T_out, nullptr, (CgScal*)nullptr, s);
    });
  });
  return rc != MPM_OK ? rc : check_launch(ctx);
}

int mpm_g2p(mpm_ctx* ctx, const void* v_hat, const void* T_hat, mpm_particles* P, void* stream) {
  if (!ctx || !v_hat || !P) return MPM_EINVAL;
  if (!ctx->have_p2g) { ctx->err = "mpm_p2g must run first"; return MPM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(ctx, [&] {
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      do_g2p<D, R>(ctx, (const R*)v_hat, (const R*)T_hat, P, s);
    });
  });
  return rc != MPM_OK ? rc : check_launch(ctx);
}

int mpm_autotune(mpm_ctx* ctx, void* stream, mpm_tuning* out) {
  if (!ctx) return MPM_EINVAL;
  if (!ctx->have_p2g) { ctx->err = "mpm_p2g must run first"; return MPM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  mpm_tuning res{};
  int rc = guarded(ctx, [&] {
    const int cand[] = {1, 2, 4, 8, 16, 32, 64};
    const int ncand = (int)(sizeof(cand) / sizeof(cand[0]));
    res.ncand = ncand;
    for (int j = 0; j < ncand; ++j) res.cand[j] = cand[j];
    if (ctx->nctile <= 0) return;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      Dev<R>& d = dev<R>(ctx);
      const R* vn = (const R*)d.gvn;
      // the Hessian's linearization at v^n (the solve forms its own from its start)
      do_surface_lin<D, R>(ctx, vn, s);
      auto op = [&](int k) {
        if (k == TUNE_ENERGY) do_energy_grad<D, R>(ctx, vn, (R*)ctx->gscratch, nullptr, SC_GT, s);
        else if (k == TUNE_HESS)
          do_hessvec<D, R>(ctx, vn, 1.0, (R*)ctx->gscratch, true, nullptr, (CgScal*)nullptr, s);
        else do_heat_apply<D, R>(ctx, (const R*)d.gTn, (R*)ctx->hr, nullptr, (CgScal*)nullptr, s);
      };
      for (int k = 0; k < TUNE_COUNT; ++k) {
        if (k == TUNE_HEAT && !ctx->p.heat) continue;
        double best = 1e300;
        int pick = 0;
        for (int j = 0; j < ncand; ++j) {
          ctx->run_tuned[k] = cand[j];
          op(k);   // warm-up
          float tmin = 1e30f;
          for (int rep = 0; rep < 3; ++rep) {
            HIPCHK(hipEventRecord(e0, s));
            op(k);
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            tmin = std::min(tmin, ms);
          }
          res.us[k][j] = 1e3 * tmin;
          if (tmin < best) { best = tmin; pick = cand[j]; }
        }
        ctx->run_tuned[k] = pick;
        res.run[k] = pick;
      }
    });
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
  });
  if (out) *out = res;
  return rc != MPM_OK ? rc : check_launch(ctx);
}

int mpm_tuning_set(mpm_ctx* ctx, const int32_t* run) {
  if (!ctx) return MPM_EINVAL;
  for (int k = 0; k < 3; ++k) ctx->run_tuned[k] = run ? std::max(0, run[k]) : 0;
  return MPM_OK;
}

int mpm_sample_surface_dev(mpm_ctx* ctx, const mpm_particles* P, double radius, double density, uint64_t seed,
                           uint64_t step, const double* label_lo, const double* label_hi, void* s_out,
                           void* dA_out, int32_t* label, int64_t cap, int64_t* out_n, void* stream) {
  if (!ctx || !P || !out_n || cap < 0 || P->n < 0 || (P->n > 0 && !P->x)) return MPM_EINVAL;
  if (cap > 0 && (!s_out || !dA_out)) return MPM_EINVAL;
  if (P->n > ctx->cap_part) { ctx->err = "more particles than the context's capacity"; return MPM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  *out_n = 0;
  int rc = guarded(ctx, [&] {
    const mpm_params& p = ctx->p;
    SmpArgs a{};
    a.n = p.n;
    a.nt = ctx->nt;
    a.dx = 1.0 / p.n;
    a.r = radius > 0 ? radius : (p.dim == 3 ? 0.867 : 0.73) * a.dx;
    a.rho = density > 0 ? density : (p.dim == 3 ? 8.0 / (a.dx * a.dx) : 4.0 / a.dx);
    if (!(a.r < a.dx)) throw ApiError{MPM_EINVAL, "sampler radius must be below dx"};
    a.key = (seed << 32) + step;
    a.has_label = label_lo && label_hi;
    for (int q = 0; q < p.dim; ++q) {
      a.lo[q] = a.has_label ? label_lo[q] : 0;
      a.hi[q] = a.has_label ? label_hi[q] : 0;
    }
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      *out_n = do_sample<D, R>(ctx, P, a, (R*)s_out, (R*)dA_out, label, cap, s);
    });
  });
  return rc != MPM_OK ? rc : check_launch(ctx);
}

int mpm_solve_momentum(mpm_ctx* ctx, void* stream) {
  if (!ctx) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(ctx, [&] {
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      if (ctx->p.krylov == MPM_KRYLOV_MINRES) do_solve_momentum_minres<D, R>(ctx, s);
      else do_solve_momentum<D, R>(ctx, s);
    });
  });
  if (rc != MPM_OK) return rc;
  rc = check_launch(ctx);
  if (rc != MPM_OK) return rc;
  return mpm_scene_status(ctx, stream);
}

int mpm_solve_heat(mpm_ctx* ctx, void* stream) {
  if (!ctx) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(ctx, [&] {
    dispatch(ctx, [&](auto Dc, auto Rv) {
      constexpr int D = decltype(Dc)::value;
      using R = decltype(Rv);
      do_solve_heat<D, R>(ctx, s);
    });
  });
  if (rc != MPM_OK) return rc;
  rc = check_launch(ctx);
  if (rc != MPM_OK) return rc;
  return mpm_scene_status(ctx, stream);
}

}  // extern "C"

namespace {

std::atomic<int> g_batch_concurrency{8};

// mpm_step_noalloc: the workspace of its context is the static device array `scratch`
// (one copy per GPU, held until the process ends), its host scalar block a static host
// array, and its context runs in single-stream mode.  Per device: the array's device
// address (taken once, with that device current), the context and a lock that orders
// the calls.
constexpr int kMaxDevices = 64;
struct NoallocSlot {
  std::mutex mu;
  bool ready = false;
  void* scratch_ptr = nullptr;
  mpm_ctx ctx;
  alignas(256) char mirror[kMirrorBytes];
};
NoallocSlot g_noalloc[kMaxDevices];

// The CFL-limited dt of the coming step (params cfl > 0), from the particles P: the
// fastest speed and, for an explicit step, the pressure-wave speed sqrt(bulk / rho_min)
// of the weakly compressible fluid; clamped to [dt_min, dt_max].  Sets the context's dt.
void choose_dt(mpm_ctx* c, const mpm_particles* P, int implicit, hipStream_t s) {
  if (!P || P->n <= 0 || !P->v || !P->m || !P->V0) throw ApiError{MPM_EINVAL, "null particle buffer"};
  unsigned long long* dv = (unsigned long long*)((char*)c->scal + kMirrorCfl);
  hipLaunchKernelGGL(k_cfl_init, dim3(1), dim3(1), 0, s, dv);
  const int nb = std::min(1024, cdiv(P->n, 256));
  dispatch(c, [&](auto Dc, auto Rv) {
    constexpr int D = decltype(Dc)::value;
    using R = decltype(Rv);
    hipLaunchKernelGGL((k_max_speed<D, R>), dim3(nb), dim3(256), 0, s, (int)P->n, (const R*)P->v, (const R*)P->m,
                       (const R*)P->V0, dv);
  });
  HIPCHK(hipGetLastError());
  read_mirror(c, s);
  const double vmax = std::sqrt(*(const double*)(c->hmirror + kMirrorCfl));
  const double rho_min = *(const double*)(c->hmirror + kMirrorCfl + 8);
  double speed = vmax;
  if (!implicit) speed = vmax + std::sqrt(c->p.bulk / rho_min);
  double dt = speed > 0 ? c->p.cfl * c->p.dx / speed : c->p.dt_max;
  dt = std::min(std::max(dt, c->p.dt_min), c->p.dt_max);
  if (!(dt > 0)) throw ApiError{MPM_EINVAL, "CFL dt not positive: dt_max must be > 0"};
  c->p.dt = dt;
  if (c->fp64) fill_params(c->d64, c->p, c->nt);
  else fill_params(c->d32, c->p, c->nt);
}

int step_one(mpm_ctx* c, mpm_particles* P, const mpm_surface* S, int implicit, hipStream_t s) {
  c->stats.host_waits = 0;
  if (c->p.cfl > 0) {
    const int rc0 = guarded(c, [&] { choose_dt(c, P, implicit, s); });
    if (rc0 != MPM_OK) return rc0;
  }
  int rc = mpm_p2g(c, P, S, s);
  c->stats.dt = c->p.dt;
  bool synced = false;   // true when the final read covered all queued work and the status
  if (rc == MPM_OK) {
    rc = guarded(c, [&] {
      dispatch(c, [&](auto Dc, auto Rv) {
        constexpr int D = decltype(Dc)::value;
        using R = decltype(Rv);
        const bool heat = c->p.heat != 0;
        CgRun run;
        hipStream_t hs = s;
        if (heat) {
          // the heat solve needs only the grid set-up: it runs on a second stream beside
          // the momentum solve
          hs = aux_fork(c, s, &c->ev_fork);
          heat_begin<D, R>(c, hs, run);
        }
        if (!implicit) do_explicit<D, R>(c, s);
        else if (c->p.krylov == MPM_KRYLOV_MINRES) do_solve_momentum_minres<D, R>(c, s);
        else do_solve_momentum<D, R>(c, s);
        if (c->p.n_planes > 0 && c->ntiles > 0) {
          // collision objects act on v^ before G2P
          Planes pl{};
          pl.n = c->p.n_planes;
          for (int k = 0; k < pl.n; ++k) {
            for (int a = 0; a < 3; ++a) { pl.o[k][a] = c->p.plane_o[k][a]; pl.nrm[k][a] = c->p.plane_n[k][a]; }
            pl.mu[k] = c->p.plane_mu[k];
          }
          const int nelem = c->ntiles * 64;
          LAUNCH(c, MPM_K_BLAS, (k_collide<D, R>), dim3(cdiv(nelem, 256)), dim3(256), 0, s,
                 (const int*)dev<R>(c).tile_list, nelem, (int)c->nn, c->nt, c->p.dx, pl, (R*)c->vhat);
        }
        if (heat) {
          heat_end<D, R>(c, hs, run);
          aux_mark(c, hs, &c->ev_join);
          aux_join(c, s, c->ev_join);
        }
        do_g2p<D, R>(c, (const R*)c->vhat, heat ? (const R*)c->That : nullptr, P, s);
        if (!implicit) {
          // an explicit step has read nothing since the binning flagged the status word
          read_mirror(c, s);
          if (c->mom_pending) {
            for (int a = 0; a < 3; ++a) c->stats.momentum[a] = a < D ? c->hbuf[SC_MOM + D + 1 + a] : 0.0;
            c->mom_pending = false;
          }
        }
        // An implicit step's Newton reads came after every kernel that flags the status
        // word, so it returns without waiting for G2P (the next step queues behind it);
        // its grid momentum is read by the next mpm_scene_status.
        synced = true;
      });
    });
  }
  if (rc == MPM_OK) rc = check_launch(c);
  int st = synced ? status_code_of(c) : mpm_scene_status(c, s);
  if (rc == MPM_OK) rc = st;
  c->stats.status = rc;
  return rc;
}

}  // namespace

extern "C" {

int mpm_batch_config(int32_t max_concurrent) {
  if (max_concurrent < 1 || max_concurrent > 64) return MPM_EINVAL;
  g_batch_concurrency = max_concurrent;
  return MPM_OK;
}

int mpm_step(mpm_ctx* const* ctxs, mpm_particles* const* P, const mpm_surface* const* S, int32_t n_scenes,
             int32_t implicit, void* stream) {
  if (!ctxs || !P || n_scenes < 0) return MPM_EINVAL;
  for (int k = 0; k < n_scenes; ++k)
    if (!ctxs[k] || !P[k]) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int> rcs(n_scenes, MPM_OK);
  const int workers = std::min<int>(g_batch_concurrency.load(), n_scenes);
  if (workers <= 1) {
    for (int k = 0; k < n_scenes; ++k) rcs[k] = step_one(ctxs[k], P[k], S ? S[k] : nullptr, implicit, s);
  } else {
    // every scene's stream starts after the work already queued on the caller's stream
    hipEvent_t ready = nullptr;
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return MPM_EHIP;
    if (hipEventRecord(ready, s) != hipSuccess) { hipEventDestroy(ready); return MPM_EHIP; }
    std::atomic<int> next{0};
    auto work = [&]() {
      for (int k = next.fetch_add(1); k < n_scenes; k = next.fetch_add(1)) {
        mpm_ctx* c = ctxs[k];
        int rc = guarded(c, [&] {
          HIPCHK(hipSetDevice(c->device));
          if (!c->own) HIPCHK(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
          if (!c->own_done) HIPCHK(hipEventCreateWithFlags(&c->own_done, hipEventDisableTiming));
          HIPCHK(hipStreamWaitEvent(c->own, ready, 0));
        });
        if (rc == MPM_OK) rc = step_one(c, P[k], S ? S[k] : nullptr, implicit, c->own);
        if (rc != MPM_EHIP && hipEventRecord(c->own_done, c->own) != hipSuccess) rc = MPM_EHIP;
        rcs[k] = rc;
      }
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < workers; ++w) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    for (int k = 0; k < n_scenes; ++k)
      if (ctxs[k]->own_done) hipStreamWaitEvent(s, ctxs[k]->own_done, 0);
    hipEventDestroy(ready);
  }
  for (int k = 0; k < n_scenes; ++k)
    if (rcs[k] != MPM_OK) return rcs[k];
  return MPM_OK;
}

int mpm_step_noalloc(const mpm_params* p, mpm_particles* P, const mpm_surface* S, int32_t implicit, void* stream,
                     size_t* scratch_bytes) {
  if (scratch_bytes) *scratch_bytes = kScratchBytes;
  if (!p || !P) return MPM_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MPM_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return MPM_EINVAL;
  NoallocSlot& sl = g_noalloc[dev];
  std::lock_guard<std::mutex> lk(sl.mu);
  mpm_ctx* c = &sl.ctx;
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(c, [&] {
    if (!sl.ready) {
      // once per device, with it current: the device address of this GPU's copy of the
      // array (host code never passes the array's own name to a kernel or a copy)
      HIPCHK(hipGetSymbolAddress(&sl.scratch_ptr, HIP_SYMBOL(scratch)));
      sl.ready = true;
    }
    const int64_t np = P->n, ns = S ? S->n : 0;
    const size_t need = workspace_need(p, np, ns);
    if (need > kScratchBytes)
      throw ApiError{MPM_ENOMEM, "mpm_step_noalloc: the scene needs " + std::to_string(need) +
                                     " bytes of workspace, the static scratch holds " + std::to_string(kScratchBytes)};
    c->single = true;
    ctx_init(c, p, sl.scratch_ptr, kScratchBytes, need, np, ns, sl.mirror, s);
  });
  if (rc == MPM_OK) rc = step_one(c, P, S, implicit, s);
  // the step is complete on the device when the call returns: the next call on this GPU
  // clears the scratch again
  if (hipStreamSynchronize(s) != hipSuccess && rc == MPM_OK) {
    c->err = "stream synchronization failed";
    rc = MPM_EHIP;
  }
  if (rc != MPM_OK) g_last_error = c->err;
  return rc;
}

int mpm_grid_view(mpm_ctx* ctx, int32_t field, void** out_ptr) {
  if (!ctx || !out_ptr) return MPM_EINVAL;
  void* p = nullptr;
  auto pick = [&](auto& d) {
    switch (field) {
      case MPM_F_MASS: p = d.gm; break;
      case MPM_F_MOM: p = d.gmv; break;
      case MPM_F_W: p = d.gW; break;
      case MPM_F_WT: p = d.gWT; break;
      case MPM_F_E: p = d.gE; break;
      case MPM_F_ET: p = d.gET; break;
      case MPM_F_VN: p = d.gvn; break;
      case MPM_F_TN: p = d.gTn; break;
      case MPM_F_FREE: p = d.gfree; break;
      case MPM_F_HEAT_RHS: p = d.hrhs; break;
      case MPM_F_HEAT_DIAG: p = d.hdiag; break;
      case MPM_F_VHAT: p = ctx->vhat; break;
      case MPM_F_THAT: p = ctx->That; break;
      case MPM_F_PARENT: p = d.s_parent_orig; break;
      case MPM_F_COUNT: p = d.pcnt_orig; break;
      case MPM_F_KSURF: p = d.sk_orig; break;
      case MPM_F_MOM_DIAG: p = d.gdiag; break;
      case MPM_F_PERM: p = d.p_perm; break;
      default: p = nullptr;
    }
  };
  if (ctx->fp64) pick(ctx->d64); else pick(ctx->d32);
  if (!p) { ctx->err = "unknown field"; return MPM_EINVAL; }
  *out_ptr = p;
  return MPM_OK;
}

int mpm_timing(mpm_ctx* ctx, int32_t enable) {
  if (!ctx) return MPM_EINVAL;
  return guarded(ctx, [&] {
    prof_collect(ctx);
    for (int k = 0; k < MPM_K_COUNT; ++k) {
      ctx->prof.ms[k] = 0;
      ctx->prof.launches[k] = 0;
      ctx->prof.dur[k].clear();
    }
    ctx->prof.on = enable != 0;
  });
}

int mpm_timing_read(mpm_ctx* ctx, double* ms, int64_t* launches, double* work_ms, int64_t* work_launches) {
  if (!ctx || !ms || !launches) return MPM_EINVAL;
  return guarded(ctx, [&] {
    prof_collect(ctx);
    for (int k = 0; k < MPM_K_COUNT; ++k) {
      ms[k] = ctx->prof.ms[k];
      launches[k] = ctx->prof.launches[k];
      double wm = 0;
      int64_t wn = 0;
      prof_work(ctx->prof, k, &wm, &wn);
      if (work_ms) work_ms[k] = wm;
      if (work_launches) work_launches[k] = wn;
    }
  });
}

int mpm_get_stats(const mpm_ctx* ctx, mpm_stats* out) {
  if (!ctx || !out) return MPM_EINVAL;
  *out = ctx->stats;
  return MPM_OK;
}

int mpm_scene_status(mpm_ctx* ctx, void* stream) {
  if (!ctx) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc = guarded(ctx, [&] {
    read_mirror(ctx, s);
    if (ctx->mom_pending) {
      const int D = ctx->p.dim;
      for (int a = 0; a < 3; ++a) ctx->stats.momentum[a] = a < D ? ctx->hbuf[SC_MOM + D + 1 + a] : 0.0;
      ctx->mom_pending = false;
    }
  });
  if (rc != MPM_OK) return rc;
  return status_code_of(ctx);
}

}  // extern "C"
