// Device kernels of the MPM hot path.  Every kernel is deterministic: integer atomics
// only build counts and slots (followed by an order fix-up), and every floating-point sum
// runs in a fixed order (node-owner gathers over cell-sorted points, fixed-tree block
// reductions, single-block final reductions).
#pragma once
#include "common.h"

namespace mpm {

// Device view of one scene's workspace.  R is double (FP64) or float (MIXED).
template <typename R>
struct Dev {
  // grid
  int n, nt, nn;
  R fn, dx, dt;
  // parameters
  R lam, mu0, mu_k, mu_T0, g0, g1, gT0, gmin, gmax, cp, K, h, T_amb, b, H;
  R gamma_label[4];
  R grav[3];
  R slab_lo[3], slab_hi[3];
  int slab, slab_axis, wall, term_mask, exact, gamma_by_label;
  // solids: phase T < T_melt (decided in FP64), Lame constants (muh0, lamh0) exp(-kh (T - Th0))
  int solids;
  double T_melt;
  R muh0, lamh0, kh, Th0;
  // point counts
  int np, ns;
  // interior particles, cell-sorted
  int* p_start; int* p_perm; int* p_key;
  R *px, *pv, *pA, *pm, *pmt, *pJ, *pV0, *pT, *pgT, *pmu, *pVn;
  R* pHc;   // Hessian coefficients: [0] dt^2 lam V0 J^2 (J term), [1] dt mu V^n (viscous)
  // solids (with d.solids): F^n [D*D][N], phase 1/0 [N], mu^h V0 and lambda^h V0 [2][N]
  R *pF, *pSol, *pLh;
  int* pcnt; int* pcnt_orig; int* grp_start; int* grp; int* gcur;
  // surface samples, cell-sorted
  int* s_start; int* s_perm; int* s_key;
  // sF: the Hessian's linearization cache, [D*D][S] surface F_r followed (with solids) by
  // [D*D][N] cof F_p of the solid particles
  R *ss, *sdA, *sk, *sk_orig, *sc, *sF;
  int* slabel; int* spar; int* s_parent_orig;
  // balance points, cell-sorted
  int* b_start; int* b_src; int* b_key; R* bx; R* bx_unsorted;
  // scratch per cell
  int* ccount;
  // grid fields
  R *gm, *gmv, *gW, *gWT, *gE, *gET, *gvn, *gTn, *gdiag, *hdiag, *hrhs;
  uint8_t* gfree;
  // tiles
  int* tile_flag; int* tile_list;
  // status, reductions
  int* status;
  double* part;
  double* scal;
};

constexpr int kPartSlot = kRedSlot;  // partial sums per reduction slot

// ======================================================================================
// Cell sort: keys, counts, slots, per-cell order fix-up.
// ======================================================================================
// Runs of equal keys among the consecutive lanes of a wave (lanes with act form a prefix
// of the wave): the lane of the run's first element and the run's length.  Points come
// in nearly cell order, so one atomic per run replaces one per point.
MPM_DEV void wave_run(int key, bool act, int& head, int& len) {
  const int lane = __lane_id();
  const int prev = __shfl_up(key, 1, kWave);
  const uint64_t heads = __ballot(act && (lane == 0 || prev != key));
  const uint64_t nact = __popcll(__ballot(act));
  const uint64_t upto = (2ull << lane) - 1;   // lanes 0..lane (all ones for lane 63)
  head = 0;
  len = 0;
  if (act) {
    head = 63 - __builtin_clzll(heads & upto);
    const uint64_t after = heads & ~upto;
    len = (after ? __builtin_ctzll(after) : (int)nact) - head;
  }
}

// Cell key of point i at x (stored in key[i]) and its count in ccount, one atomic per run
// of equal keys in the wave.  Every lane of the wave calls it (act: the lane has a point).
template <int D, typename R>
MPM_DEV void cell_key_count(const R* x, bool act, int i, int n, int nt, R fn, int* key, int* ccount, int* status) {
  int k = 0;
  if (act) {
    int c[D]; R f[D]; bool bad = false;
    locate<D, R>(x, n, fn, c, f, &bad);
    if (bad) flag_status(status, ST_DOMAIN);
    k = (int)tiled_index<D>(c, nt);
    key[i] = k;
  }
  int head, len;
  wave_run(k, act, head, len);
  if (act && __lane_id() == head) atomicAdd(&ccount[k], len);
}

template <int D, typename R>
__global__ void k_cell_keys(const R* pos, int cnt, int n, int nt, R fn, int* key, int* ccount, int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < cnt;
  R x[D];
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = act ? pos[(int64_t)a * cnt + i] : R(0);
  cell_key_count<D, R>(x, act, i, n, nt, fn, key, ccount, status);
}

constexpr int kScanT = 256, kScanI = 16, kScanBlock = kScanT * kScanI;
constexpr int kScanSpin = 1 << 22;   // polls of one look-back window before giving up

// Status word of a scan block: value | state << 32 | epoch << 34, state 1 = the block's
// own sum, 2 = its inclusive prefix.  Words of an earlier scan carry another epoch.
MPM_DEV uint64_t scan_word(unsigned epoch, unsigned state, unsigned value) {
  return (uint64_t)value | ((uint64_t)state << 32) | ((uint64_t)epoch << 34);
}

// Sum over the wave, in every lane.
MPM_DEV int wave_sum_all(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Single-pass exclusive scan of in[0,len) into out[0,len), out[len] = total.  Block b
// scans kScanBlock elements; it publishes its sum at once, then wave 0 reads the status
// words of up to 64 predecessors at a time, going back until it meets an inclusive prefix
// (block 0 publishes one at once), and publishes its own.  Workgroups start in index order,
// so every predecessor is running or done and each wait ends; the wait is still bounded:
// after kScanSpin polls without progress the block flags ST_STALL and the scan is invalid.
__global__ void __launch_bounds__(kScanT) k_scan(const int* in, int* out, int len, uint64_t* flags, unsigned epoch,
                                                 int* status) {
  __shared__ int wsum[kScanT / kWave];
  __shared__ int excl;
  const int b = blockIdx.x, t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
  const int base = b * kScanBlock + t * kScanI;
  int v[kScanI];
  if (base + kScanI <= len) {
    const int4* p4 = (const int4*)(in + base);
#pragma unroll
    for (int q = 0; q < kScanI / 4; ++q) {
      int4 x = p4[q];
      v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanI; ++k) v[k] = base + k < len ? in[base + k] : 0;
  }
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanI; ++k) s += v[k];
  int incl = s;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  int woff = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kScanT / kWave; ++w) {
    int x = wsum[w];
    woff += w < wid ? x : 0;
    total += x;
  }
  if (wid == 0) {
    if (b == 0) {
      if (lane == 0) {
        __hip_atomic_store(flags, scan_word(epoch, 2, (unsigned)total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        excl = 0;
      }
    } else {
      if (lane == 0)
        __hip_atomic_store(flags + b, scan_word(epoch, 1, (unsigned)total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int prefix = 0, top = b - 1, spins = 0;
      bool stalled = false;
      for (;;) {
        const int idx = top - lane;
        uint64_t w = idx >= 0 ? __hip_atomic_load(flags + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        const unsigned st = (unsigned)(w >> 32) & 3u;
        const bool ready = idx < 0 || ((unsigned)(w >> 34) == epoch && st != 0);
        const uint64_t waiting = __ballot(!ready);
        const uint64_t pref = __ballot(idx >= 0 && ready && st == 2);
        const int pl = pref ? __builtin_ctzll(pref) : kWave;             // nearest prefix
        const uint64_t upto = pl == kWave ? ~0ull : (2ull << pl) - 1;   // lanes 0..pl
        if ((waiting & upto) == 0) {
          prefix += wave_sum_all(lane <= pl && idx >= 0 ? (int)(unsigned)w : 0);
          if (pl < kWave) break;
          top -= kWave;
          spins = 0;
          continue;
        }
        if (++spins > kScanSpin) { stalled = true; break; }
        __builtin_amdgcn_s_sleep(1);
      }
      if (lane == 0) {
        if (stalled) flag_status(status, ST_STALL);
        __hip_atomic_store(flags + b, scan_word(epoch, 2, (unsigned)(prefix + total)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        excl = prefix;
      }
    }
  }
  __syncthreads();
  int run = excl + woff + incl - s;
  if (base + kScanI <= len) {
    int4* o4 = (int4*)(out + base);
#pragma unroll
    for (int q = 0; q < kScanI / 4; ++q) {
      int4 x;
      x.x = run; run += v[4 * q];
      x.y = run; run += v[4 * q + 1];
      x.z = run; run += v[4 * q + 2];
      x.w = run; run += v[4 * q + 3];
      o4[q] = x;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanI; ++k) {
      if (base + k < len) out[base + k] = run;
      run += v[k];
    }
  }
  if (b == (int)gridDim.x - 1 && t == kScanT - 1) out[len] = excl + total;
}

// Slots from the remaining cell count: a run of len equal keys takes the len slots below
// start[key] + (count before its atomic), in input order.  Leaves the counters at zero.
__global__ void k_cell_scatter(const int* key, int cnt, const int* start, int* ccount, int* perm, int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < cnt;
  const int k = act ? key[i] : 0;
  int head, len;
  wave_run(k, act, head, len);
  const int lane = __lane_id();
  int rem = 0;
  if (act && lane == head) rem = atomicSub(&ccount[k], len);
  rem = __shfl(rem, head, kWave);
  if (act) {
    const int slot = start[k] + rem - len + (lane - head);
    if (slot >= 0 && slot < cnt) perm[slot] = i;
    else flag_status(status, ST_INTERNAL);
  }
}

// Segment ordering after an atomic scatter, from src into dst: the segment of slot s is
// the run of slots whose values v have the same key[v]; it starts at start[key[v]].
// Sorting each segment by value (the input index) puts it in input order, independent of
// the order in which the atomics were served.  Every thread ranks its own value by
// counting the smaller ones in its segment (independent loads; the values are distinct).
// src is only read, so every thread sees the scatter's output.

__global__ void k_segment_order(const int* key, const int* start, int cnt, const int* src, int* dst) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  const int v = src[s];
  const int k = key[v];
  const int b = start[k], e = start[k + 1], n = e - b;
  if (n < 2) {
    dst[s] = v;
    return;
  }
  // the rank of v among its segment's (distinct) values, found by this thread alone
  int r = 0;
  for (int j = b; j < e; ++j) r += src[j] < v ? 1 : 0;
  dst[b + r] = v;
}

__global__ void k_fill_i32(int* p, int v, int64_t len) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = v;
}

template <typename R>
__global__ void k_fill_r(R* p, R v, int64_t len) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = v;
}

// ======================================================================================
// Particle and sample staging in cell order.
// ======================================================================================
template <int D, typename R>
__global__ void k_gather_particles(Dev<R> d, const R* x, const R* v, const R* A, const R* J,
                                   const R* V0, const R* m, const R* T, const R* gT, const R* F) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int N = d.np;
  if (k >= N) return;
  int i = d.p_perm[k];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    d.px[a * N + k] = x[a * N + i];
    d.pv[a * N + k] = v[a * N + i];
    d.pgT[a * N + k] = gT[a * N + i];
  }
#pragma unroll
  for (int a = 0; a < D * D; ++a) d.pA[a * N + k] = A[a * N + i];
  R Jk = J[i], V0k = V0[i], Tk = T[i];
  d.pJ[k] = Jk;
  d.pV0[k] = V0k;
  d.pm[k] = m[i];
  d.pT[k] = Tk;
  const R Vn = Jk * V0k;
  R mu = d.mu0 == R(0) ? R(0) : d.mu0 * exp(-d.mu_k * (Tk - d.mu_T0));
  bool sol = false;
  if (d.solids) {
    // a solid has no fluid pressure and no viscosity
    sol = (double)Tk < d.T_melt;
    d.pSol[k] = sol ? R(1) : R(0);
    const R fh = exp(-d.kh * (Tk - d.Th0));
    d.pLh[k] = sol ? d.muh0 * fh * V0k : R(0);
    d.pLh[N + k] = sol ? d.lamh0 * fh * V0k : R(0);
#pragma unroll
    for (int a = 0; a < D * D; ++a) d.pF[a * N + k] = F[a * N + i];
    if (sol) mu = R(0);
  }
  d.pVn[k] = Vn;
  d.pmu[k] = mu;
  // the Hessian's per-particle factors, rounded as the Hessian kernel would form them
  d.pHc[k] = sol ? R(0) : d.dt * d.dt * d.lam * V0k * Jk * Jk;
  d.pHc[N + k] = d.dt * (mu * Vn);
  d.pcnt[k] = 0;
}

template <int D, typename R>
__global__ void k_gather_surface(Dev<R> d, const R* s, const R* dA, const int* label) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int S = d.ns;
  if (k >= S) return;
  int i = d.s_perm[k];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    d.ss[a * S + k] = s[a * S + i];
    d.sdA[a * S + k] = dA[a * S + i];
  }
  d.slabel[k] = label ? label[i] : 0;
}

// Squared distance in double with separate roundings (no contraction), summed axis by
// axis: the same arithmetic any reference evaluating ((d0^2 + d1^2) + d2^2) performs.
template <int D>
MPM_DEV double dist2_exact(const double* a, const double* b) {
  double acc = mul_nc(a[0] - b[0], a[0] - b[0]);
#pragma unroll
  for (int k = 1; k < D; ++k) acc = add_nc(acc, mul_nc(a[k] - b[k], a[k] - b[k]));
  return acc;
}

// Nearest interior particle of sample r (Section 4.1.2); ties to the lower input index.
// Searches the cells within 1, 2, then 3 cells of the sample; a winner closer than the
// searched radius (rad * dx) is exact, since every particle outside the searched block
// is at least that far.  Otherwise falls back to a scan of all particles.  Returns the
// sorted index and its input index.
template <int D, typename R>
MPM_DEV int parent_search(const Dev<R>& d, const double* sd, const int* c, int& borig_out) {
  const int N = d.np;
  double best = 1e300;
  int bk = -1, borig = -1;   // borig: input index of bk, loaded only when a tie needs it
  auto visit = [&](int k) {
    double xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = (double)d.px[a * N + k];
    double d2 = dist2_exact<D>(sd, xp);
    if (d2 < best) {
      best = d2; bk = k; borig = -1;
    } else if (d2 == best) {
      if (borig < 0) borig = d.p_perm[bk];
      int o = d.p_perm[k];
      if (o < borig) { bk = k; borig = o; }
    }
  };
  double dxd = (double)d.dx;
  // own cell first, so that the box test below prunes most neighbours
  {
    int ci = (int)tiled_index<D>(c, d.nt);
    for (int k = d.p_start[ci]; k < d.p_start[ci + 1]; ++k) visit(k);
  }
  for (int rad = 1; rad <= 3; ++rad) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) { lo[a] = max(c[a] - rad, 0); hi[a] = min(c[a] + rad, d.n - 1); }
    for (int z = (D == 3 ? lo[2] : 0); z <= (D == 3 ? hi[2] : 0); ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          int cc[3] = {x, y, z};
          // shell rad only: inner cells were searched by the smaller radii
          int ring = 0;
          double bd2 = 0;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            ring = max(ring, abs(cc[a] - c[a]));
            double lo_a = cc[a] * dxd, hi_a = (cc[a] + 1) * dxd;
            double g = sd[a] < lo_a ? lo_a - sd[a] : (sd[a] > hi_a ? sd[a] - hi_a : 0.0);
            bd2 += g * g;
          }
          if (ring != rad) continue;
          // no point of the cell can be closer than its box; the margin keeps the test
          // conservative against the rounding of both distances (ties must be visited)
          if (bd2 > best * (1.0 + 1e-9)) continue;
          int ci = (int)tiled_index<D>(cc, d.nt);
          for (int k = d.p_start[ci]; k < d.p_start[ci + 1]; ++k) visit(k);
        }
    if (best < (rad * dxd) * (rad * dxd)) break;
    if (rad == 3) {
      best = 1e300; bk = -1; borig = -1;
      for (int k = 0; k < N; ++k) visit(k);
    }
  }
  if (bk >= 0 && borig < 0) borig = d.p_perm[bk];
  borig_out = borig;
  return bk;
}

// Parents of the samples, a group of kParGroup lanes per sample, ring by ring as in
// parent_search: the lanes share the particles of the sample's own cell, then the cells
// of ring 1 and, if needed, ring 2 (cells at Chebyshev distance 1, 2 from the sample's
// cell), each skipped when its box is farther than the group's best so far (the cells the
// sequential search prunes).  The group takes the minimum of (distance, input index), a
// total order, so the result is the sequential search's.  After ring rad a winner closer
// than rad dx is exact; past ring 2 the group's first lane runs the sequential search.
constexpr int kParGroup = 8;

// The cells of rings 1 and 2 around a cell (Chebyshev distance 1, then 2), each as its
// index j in the 5^D block of offsets -2..2 (offset a = j / 5^a % 5 - 2): ring 1 in
// off[0, n1), ring 2 in off[n1, n1 + n2).
template <int D>
struct RingCells {
  int n1 = 0, n2 = 0;
  int off[D == 3 ? 124 : 24] = {};
  constexpr RingCells() {
    const int nb = D == 3 ? 125 : 25;
    for (int ring = 1; ring <= 2; ++ring)
      for (int j = 0; j < nb; ++j) {
        const int o0 = j % 5 - 2, o1 = (j / 5) % 5 - 2, o2 = D == 3 ? j / 25 - 2 : 0;
        const int a0 = o0 < 0 ? -o0 : o0, a1 = o1 < 0 ? -o1 : o1, a2 = o2 < 0 ? -o2 : o2;
        const int r = a0 > a1 ? (a0 > a2 ? a0 : a2) : (a1 > a2 ? a1 : a2);
        if (r != ring) continue;
        if (ring == 1) off[n1++] = j;
        else off[n1 + n2++] = j;
      }
  }
};
__constant__ RingCells<2> kRing2 = RingCells<2>();
__constant__ RingCells<3> kRing3 = RingCells<3>();

template <int D>
MPM_DEV void par_min(double& best, int& bk, const int* perm) {
#pragma unroll
  for (int o = kParGroup / 2; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, kParGroup);
    const int ok = __shfl_xor(bk, o, kParGroup);
    bool take = ob < best;
    if (!take && ob == best && ok >= 0 && bk >= 0 && ok != bk) take = perm[ok] < perm[bk];
    if (take) { best = ob; bk = ok; }
  }
}

template <int D, typename R>
__global__ void __launch_bounds__(256) k_parents(Dev<R> d) {
  const int lane = threadIdx.x & (kParGroup - 1);
  const int r = blockIdx.x * (256 / kParGroup) + threadIdx.x / kParGroup;
  const int S = d.ns, N = d.np;
  const bool live = r < S;
  double sd[D];
  int c[D];
  if (live) {
    R sr[D], f[D];
#pragma unroll
    for (int a = 0; a < D; ++a) { sr[a] = d.ss[a * S + r]; sd[a] = (double)sr[a]; }
    bool bad = false;
    locate<D, R>(sr, d.n, d.fn, c, f, &bad);
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) { sd[a] = 0; c[a] = 0; }
  }
  double best = 1e300;
  int bk = -1, bo = -1;
  auto visit = [&](int k) {
    double xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = (double)d.px[a * N + k];
    const double d2 = dist2_exact<D>(sd, xp);
    if (d2 < best) {
      best = d2; bk = k; bo = -1;
    } else if (d2 == best) {
      if (bo < 0) bo = d.p_perm[bk];
      const int o = d.p_perm[k];
      if (o < bo) { bk = k; bo = o; }
    }
  };
  if (live) {
    const int ci = (int)tiled_index<D>(c, d.nt);
    for (int k = d.p_start[ci] + lane; k < d.p_start[ci + 1]; k += kParGroup) visit(k);
  }
  par_min<D>(best, bk, d.p_perm);
  const double dxd = (double)d.dx;
  bool done = false;
  const RingCells<D>& rings = *(D == 3 ? (const RingCells<D>*)&kRing3 : (const RingCells<D>*)&kRing2);
  for (int rad = 1; rad <= 2 && !done; ++rad) {
    constexpr int W = 5;                                  // offsets -2..2 per axis
    const double cut = best * (1.0 + 1e-9);                // ties must be visited
    const int q0 = rad == 1 ? 0 : rings.n1, q1 = rad == 1 ? rings.n1 : rings.n1 + rings.n2;
    for (int q = q0 + lane; live && q < q1; q += kParGroup) {
      const int j = rings.off[q];
      const int o0 = j % W - 2, o1 = (j / W) % W - 2, o2 = D == 3 ? j / (W * W) - 2 : 0;
      int cc[3] = {c[0] + o0, c[1] + o1, D == 3 ? c[2] + o2 : 0};
      bool in = true;
      double bd2 = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        in = in && cc[a] >= 0 && cc[a] < d.n;
        const double lo_a = cc[a] * dxd, hi_a = (cc[a] + 1) * dxd;
        const double g = sd[a] < lo_a ? lo_a - sd[a] : (sd[a] > hi_a ? sd[a] - hi_a : 0.0);
        bd2 += g * g;
      }
      if (in && !(bd2 > cut)) {
        const int ci = (int)tiled_index<D>(cc, d.nt);
        for (int k = d.p_start[ci]; k < d.p_start[ci + 1]; ++k) visit(k);
      }
    }
    par_min<D>(best, bk, d.p_perm);
    done = bk >= 0 && best < (rad * dxd) * (rad * dxd);
  }
  if (!live || lane != 0) return;
  int borig = -1;
  if (!done) bk = parent_search<D, R>(d, sd, c, borig);
  if (bk < 0) { flag_status(d.status, ST_DOMAIN); bk = 0; }
  if (borig < 0) borig = d.p_perm[bk];
  d.spar[r] = bk;
  d.s_parent_orig[d.s_perm[r]] = borig;
  atomicAdd(&d.pcnt[bk], 1);
}

// m~_p = m_p / (2 |Pi_p| + 1) (Section 4.1.3); cursor copy for the group CSR.
template <typename R>
__global__ void k_split_mass(Dev<R> d) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.np) return;
  int c = d.pcnt[k];
  d.pmt[k] = d.pm[k] / (R(2) * R(c) + R(1));
  d.gcur[k] = c;
  d.pcnt_orig[d.p_perm[k]] = c;
}

// Balance point b_r = s_r + 2 (x_p(r) - s_r) (eq. pbal), in sample order, with its cell
// key and count (the first step of its cell sort); group slots (each group in atomic
// order, put in sample order by k_segment_order).
template <int D, typename R>
__global__ void k_balance(Dev<R> d, int* grp_unordered) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int S = d.ns, N = d.np;
  const bool act = r < S;
  R b[D];
#pragma unroll
  for (int a = 0; a < D; ++a) b[a] = R(0);
  if (act) {
    const int p = d.spar[r];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const R s = d.ss[a * S + r];
      b[a] = s + R(2) * (d.px[a * N + p] - s);
      d.bx_unsorted[a * S + r] = b[a];
    }
    const int slot = d.grp_start[p] + atomicSub(&d.gcur[p], 1) - 1;
    grp_unordered[slot] = r;
  }
  cell_key_count<D, R>(b, act, r, d.n, d.nt, d.fn, d.b_key, d.ccount, d.status);
}

template <int D, typename R>
__global__ void k_gather_balance(Dev<R> d) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int S = d.ns;
  if (k >= S) return;
  int r = d.b_src[k];
#pragma unroll
  for (int a = 0; a < D; ++a) d.bx[a * S + k] = d.bx_unsorted[a * S + r];
}

// Marks the tiles that hold a node of any occupied cell's stencil.
template <int D, typename R>
__global__ void k_mark_tiles(Dev<R> d) {
  int ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= d.nn) return;
  int occ = (d.p_start[ci + 1] - d.p_start[ci]) + (d.ns ? (d.s_start[ci + 1] - d.s_start[ci]) + (d.b_start[ci + 1] - d.b_start[ci]) : 0);
  if (occ == 0) return;
  int c[3] = {0, 0, 0};
  tiled_coords<D>(ci / kTileNodes, ci % kTileNodes, d.nt, c);
  constexpr int L = Tiling<D>::LOG;
  int tlo[3] = {0, 0, 0}, thi[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    tlo[a] = max(c[a] - 1, 0) >> L;
    thi[a] = min(c[a] + 1, d.n - 1) >> L;
  }
  for (int t2 = tlo[2]; t2 <= thi[2]; ++t2)
    for (int t1 = tlo[1]; t1 <= thi[1]; ++t1)
      for (int t0 = tlo[0]; t0 <= thi[0]; ++t0) {
        int t = t0 + d.nt * (t1 + (D == 3 ? d.nt * t2 : 0));
        d.tile_flag[t] = 1;
      }
}

__global__ void k_compact_tiles(const int* flag, const int* pos, int ntile, int* list) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntile && flag[t]) list[pos[t]] = t;
}

// Zeroes every grid field on the listed tiles and clears their flags.
template <int D, typename R>
__global__ void k_clear_tiles(Dev<R> d, const int* list, R* const* extra, int nextra, int ncomp_extra) {
  int t = list[blockIdx.x];
  int node = t * kTileNodes + threadIdx.x;
  int nn = d.nn;
  d.gm[node] = 0; d.gW[node] = 0; d.gWT[node] = 0; d.gE[node] = 0; d.gET[node] = 0;
  d.gTn[node] = 0; d.hdiag[node] = 0; d.hrhs[node] = 0; d.gfree[node] = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    d.gmv[a * nn + node] = 0; d.gvn[a * nn + node] = 0; d.gdiag[a * nn + node] = 0;
  }
  for (int e = 0; e < nextra; ++e)
    for (int a = 0; a < ncomp_extra; ++a) extra[e][a * nn + node] = 0;
  if (threadIdx.x == 0) d.tile_flag[t] = 0;
}

// k_r = gamma(T^s_r), T^s_r = sum_i N_i(s_r) T^n_i (Section 4.3.1), or by label (Sec. 3.6);
// gamma_by_label 2: gamma(T^s_r) on the free surface (label 1), gamma_label[0] elsewhere.
template <int D, typename R>
__global__ void k_surface_k(Dev<R> d) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  int S = d.ns;
  if (r >= S) return;
  R kr;
  if (d.gamma_by_label == 1) {
    int l = d.slabel[r];
    kr = d.gamma_label[l & 3];
  } else if (d.gamma_by_label == 2 && d.slabel[r] != 1) {
    kr = d.gamma_label[0];   // a sample against the container's walls
  } else {
    R x[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = d.ss[a * S + r];
    Stencil<D, R> st; bool bad = false;
    make_stencil<D, R>(x, d.n, d.fn, st, &bad);
    R Ts = 0;
    for_stencil<D>([&](int k0, int k1, int k2) {
      int nd[3] = {st.c[0] - 1 + k0, st.c[1] - 1 + k1, D == 3 ? st.c[2] - 1 + k2 : 0};
      R g[D];
      R Nw = node_weight<D, R>(st, k0, k1, k2, g);
      Ts += Nw * d.gTn[tiled_index<D>(nd, d.nt)];
    });
    kr = d.g0 + d.g1 * (Ts - d.gT0);
    kr = kr < d.gmin ? d.gmin : (kr > d.gmax ? d.gmax : kr);
  }
  d.sk[r] = kr;
  d.sk_orig[d.s_perm[r]] = kr;
}

// ======================================================================================
// Energy, gradient and Hessian-vector product (Section 4.3.1).  Point phase: every
// quadrature point gathers the velocity (or direction) gradient from its stencil and
// forms a stress-like matrix S_q; node phase: every node gathers sum_q S_q grad N_i(x_q).
// ======================================================================================
enum PointMode { PM_ENERGY = 0, PM_HESS = 1 };

// Gradient sum_j u_j (x) grad N_j at a stencil; optional projection by the free mask.
template <int D, typename R>
MPM_DEV void gather_grad(const Dev<R>& d, const Stencil<D, R>& st, const R* u, bool mask, R (&G)[D][D]) {
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) G[a][b] = 0;
  for_stencil<D>([&](int k0, int k1, int k2) {
    int nd[3] = {st.c[0] - 1 + k0, st.c[1] - 1 + k1, D == 3 ? st.c[2] - 1 + k2 : 0};
    int node = (int)tiled_index<D>(nd, d.nt);
    R g[D];
    node_weight<D, R>(st, k0, k1, k2, g);
    uint8_t fr = mask ? d.gfree[node] : 0xff;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R ua = (fr >> a) & 1 ? u[a * d.nn + node] : R(0);
#pragma unroll
      for (int b = 0; b < D; ++b) G[a][b] += ua * g[b];
    }
  });
}

template <typename R>
MPM_DEV void cross3(const R* u, const R* v, R* w) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}

enum NodeMode { NM_GRAD = 0, NM_HESS = 1 };

// ======================================================================================
// G2P with merge (Section 5).
// ======================================================================================
// Interpolated velocity and first moment about ref: sum_i N_i(q) v^_i and
// sum_i N_i(q) v^_i (x_i - ref)^T, with x_i - ref = (x_i - q) + (q - ref).
template <int D, typename R>
MPM_DEV void g2p_moments(const Dev<R>& d, const R* q, const R* qref, const R* vh, R* vq, R (&tq)[D][D]) {
  Stencil<D, R> st; bool bad = false;
  make_stencil<D, R>(q, d.n, d.fn, st, &bad);
#pragma unroll
  for (int a = 0; a < D; ++a) { vq[a] = 0; for (int b = 0; b < D; ++b) tq[a][b] = 0; }
  R shift[D];
#pragma unroll
  for (int a = 0; a < D; ++a) shift[a] = q[a] - qref[a];
  for_stencil<D>([&](int k0, int k1, int k2) {
    int kk[3] = {k0, k1, k2};
    int nd[3] = {st.c[0] - 1 + k0, st.c[1] - 1 + k1, D == 3 ? st.c[2] - 1 + k2 : 0};
    int node = (int)tiled_index<D>(nd, d.nt);
    R g[D];
    R Nw = node_weight<D, R>(st, k0, k1, k2, g);
    R rel[D];
#pragma unroll
    for (int b = 0; b < D; ++b) rel[b] = (R(kk[b]) - R(0.5) - st.f[b]) * d.dx + shift[b];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R nv = Nw * vh[a * d.nn + node];
      vq[a] += nv;
#pragma unroll
      for (int b = 0; b < D; ++b) tq[a][b] += nv * rel[b];
    }
  });
}

// Per sample r: v(s_r) + v(b_r) and the first moments of both about x_p(r).
template <int D, typename R>
__global__ void k_g2p_split(Dev<R> d, const R* vh) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int S = d.ns, N = d.np;
  if (r >= S) return;
  int p = d.spar[r];
  R xp[D], s[D], b[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xp[a] = d.px[a * N + p];
    s[a] = d.ss[a * S + r];
    b[a] = s[a] + R(2) * (xp[a] - s[a]);
  }
  R v1[D], v2[D], t1[D][D], t2[D][D];
  g2p_moments<D, R>(d, s, xp, vh, v1, t1);
  g2p_moments<D, R>(d, b, xp, vh, v2, t2);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    d.sc[a * S + r] = v1[a] + v2[a];
#pragma unroll
    for (int c = 0; c < D; ++c) d.sc[(D + a * D + c) * S + r] = t1[a][c] + t2[a][c];
  }
}

// ======================================================================================
// Krylov BLAS-1 over the nodes of the active tiles (ncomp components, dense arrays of nn
// per component).  Grid-stride with a fixed grid, so the partial-sum partition depends
// only on the problem size.
// ======================================================================================
struct CgScal {
  double rz, rr, pAp, tol2, alpha, beta, rz0, spare;
  int done, iters, maxit, breakdown;
};

// Reduction counters (one per reduction site; each returns to zero after use).
// Reduction counter sites.  The heat solve has its own sites (CTR_H*) so that it can run
// on a second stream concurrently with the momentum solve.
enum : int {
  CTR_DOT = 0, CTR_MOM = 1, CTR_CGSTART = 2, CTR_MERGE = 3, CTR_CGUPD = 4,
  CTR_HSTART = 5, CTR_HUPD = 6, CTR_HMERGE = 7, CTR_HDOT = 8, CTR_COUNT = 12
};

MPM_DEV int elem_node(const int* tile_list, int e) { return tile_list[e >> 6] * kTileNodes + (e & 63); }

// Most components of a node vector (D velocity components, or 1 temperature).  The node
// kernels load all of a node's components before they store any: for the compiler a
// store may alias a later load, which would otherwise wait for it.
constexpr int kMaxComp = 3;

// Threads of a block of the node kernels below (their multi-value block sums hold
// NV x kNodeThreads doubles of LDS).
constexpr int kNodeThreads = 256;

// dst = sum over the active nodes of a . b (ncomp components), reduced in fixed order.
template <typename R>
__global__ void k_dot(const int* tl, int nelem, int nn, int ncomp, const R* a, const R* b, double* part,
                      unsigned* ctr, double* dst) {
  __shared__ double sh[kRedSh];
  double s = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    for (int c = 0; c < ncomp; ++c) s += (double)a[c * nn + node] * (double)b[c * nn + node];
  }
  double t = block_sum(s, sh), r;
  if (grid_reduce<1>(&t, part, ctr, sh, &r) && threadIdx.x == 0) *dst = r;
}

// Sums nslot partial arrays of nb entries each (fixed order) into dst[0..nslot).
__global__ void k_finalize(const double* part, int nb, int nslot, double* dst) {
  __shared__ double sh[kRedSh];
  for (int s = 0; s < nslot; ++s) {
    double v = 0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) v += part[s * kPartSlot + k];
    double t = block_sum(v, sh);
    if (threadIdx.x == 0) dst[s] = t;
    __syncthreads();
  }
}

// Input update fused into an operator application: the operator is applied to z + beta u
// instead of u (its tile kernel forms the values it stages, its node kernel forms its
// nodes' values and stores them in p).  Used for the CG direction p = z + beta p (p == u,
// beta from the CG scalars, 0 before the first update so that p = z) and for the line-
// search trial v^ + alpha delta (u = delta, beta = alpha given by the host, p = the trial
// point).  z == nullptr: no update.
template <typename R>
struct PUpd {
  R* p;
  const R* z;
  const CgScal* cg;   // beta = cg->beta; nullptr: beta = beta_h
  R beta_h;
  MPM_DEV R beta() const { return z ? (cg ? (R)cg->beta : beta_h) : R(0); }
};

// The new direction z + beta p, contracted explicitly so that the operator's two kernels
// form it bitwise alike.
MPM_DEV float cg_dir(float z, float beta, float p) { return __builtin_fmaf(beta, p, z); }
MPM_DEV double cg_dir(double z, double beta, double p) { return __builtin_fma(beta, p, z); }

// CG scalars from the sums r.z, r.r of the starting residual.
MPM_DEV void cg_init(CgScal* s, double rz, double rr, double tol2, int maxit) {
  s->beta = 0;
  s->rz = rz;
  s->rr = rr;
  s->tol2 = tol2;
  s->maxit = maxit;
  s->iters = 0;
  s->breakdown = 0;
  s->done = (rr <= tol2) || maxit <= 0 || !(rr == rr) || rr > 1e300;
}

// Start of a CG solve for the right side bscale * b: r = bscale b - A x0 (Ax = null: x0 = 0
// and x is zeroed), z = r / diag,
// p = z; the last block sets the scalars.  tol2 = tol2_host * (*tol2_scale) if given.
template <typename R>
__global__ void k_cg_start(const int* tl, int nelem, int nn, int ncomp, const R* b, R bscale, const R* Ax,
                           const R* diag, R* x, R* r, R* z, R* p, double* part, unsigned* ctr, CgScal* cs,
                           double tol2_host, const double* tol2_scale, int maxit, const double* gate) {
  __shared__ double sh[2 * kNodeThreads];
  if (gate && *gate == 0.0) return;   // a speculative start that was called off
  double rz = 0, rr = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    R bv[kMaxComp], av[kMaxComp], dv[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      bv[c] = b[j];
      av[c] = Ax ? Ax[j] : R(0);
      dv[c] = diag[j];
    }
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      R rv = Ax ? bscale * bv[c] - av[c] : bscale * bv[c];
      R zv = rv / dv[c];
      if (!Ax) x[j] = 0;
      r[j] = rv; z[j] = zv; p[j] = zv;
      rz += (double)rv * (double)zv;
      rr += (double)rv * (double)rv;
    }
  }
  double v[2] = {rz, rr}, t[2], sum[2];
  block_sum_n<2>(v, sh, t);
  if (grid_reduce<2>(t, part, ctr, sh, sum) && threadIdx.x == 0)
    cg_init(cs, sum[0], sum[1], tol2_host * (tol2_scale ? *tol2_scale : 1.0), maxit);
}

// Whether the Newton iteration after the current trial follows at once, decided on the
// device from the trial's sums with the host's tests (the Armijo test at alpha = 1 with
// its round-off allowance, then the stopping tests at the new iterate): writes 1 or 0 to
// scal[go_slot], and the CG tolerance max(cg_rel |g|, 0.1 newton_tol |g0|)^2 of that
// iteration to scal[tol_slot].  from_start: the current iterate is the start, whose
// values come from the start's sums at scal[g0_slot] instead of the host's.
// scal == nullptr: no decision.
struct NewtonDecide {
  double* scal;
  int dim, gt_slot, g0_slot, from_start;
  double phi_h, g0_h, floor_h, gcur_h, c1, eps8;
  int armijo;
  double newton_tol, cg_rel;
  int mixed;
  double dx_over_dt;
  int go_slot, tol_slot;
};

MPM_DEV bool newton_decide(const NewtonDecide& a) {
  double* scal = a.scal;
  const int dim = a.dim;
  double phi = a.phi_h, g0 = a.g0_h, floor_abs = a.floor_h, gcur = a.gcur_h;
  if (a.from_start) {
    phi = scal[a.g0_slot];
    g0 = sqrt(fmax(scal[a.g0_slot + dim + 2], 0.0));
    floor_abs = 1e-14 * scal[a.g0_slot + 1 + dim] * a.dx_over_dt;
    gcur = g0;
  }
  const double phit = scal[a.gt_slot], slope = scal[a.gt_slot + dim + 3];
  const double gn = sqrt(fmax(scal[a.gt_slot + dim + 2], 0.0));
  const bool start_ok = g0 == g0 && phi == phi && !(g0 <= fmax(a.newton_tol * g0, floor_abs));
  const bool accept = !a.armijo || phit <= phi + a.c1 * slope + a.eps8 * fmax(fabs(phi), fabs(phit));
  // the MIXED stop as the host takes it: |g| below 1e-4 |g0| or below eps32 times the size
  // of the gradient's terms (sums slot dim+4), and not halved by the step
  const double fl32 = 1.1920928955078125e-07 * sqrt(fmax(scal[a.gt_slot + dim + 4], 0.0));
  const bool go = start_ok && accept && gn == gn && phit == phit && !(gn <= fmax(a.newton_tol * g0, floor_abs)) &&
                  !(a.mixed && (gn <= 1e-4 * g0 || gn <= fl32) && gn > 0.5 * gcur);
  const double t = fmax(a.cg_rel * gn, 0.1 * a.newton_tol * g0);
  scal[a.go_slot] = go ? 1.0 : 0.0;
  scal[a.tol_slot] = t * t;
  return go;
}

// The decision alone (one thread); when the iteration does not follow, the next CG's
// scalars are marked done so that a CG queued for it returns at once.
__global__ void k_newton_decide(NewtonDecide a, CgScal* next) {
  if (!newton_decide(a)) next->done = 1;
}

// Called by the last block of the operator's merge with the sum p . A p.
MPM_DEV void cg_set_alpha(CgScal* s, double pAp) {
  if (s->done) return;
  s->pAp = pAp;
  if (!(pAp > 0.0)) { s->done = 1; s->breakdown = 1; return; }
  s->alpha = s->rz / pAp;
}

template <typename R>
__global__ void k_cg_update(const int* tl, int nelem, int nn, int ncomp, CgScal* s, R* x, R* r, R* z,
                            const R* p, const R* Ap, const R* diag, double* part, unsigned* ctr) {
  __shared__ double sh[2 * kNodeThreads];
  if (s->done) return;
  R alpha = (R)s->alpha;
  double rz = 0, rr = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    R xv[kMaxComp], pv[kMaxComp], rv0[kMaxComp], av[kMaxComp], dv[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      xv[c] = x[j]; pv[c] = p[j]; rv0[c] = r[j]; av[c] = Ap[j]; dv[c] = diag[j];
    }
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      x[j] = xv[c] + alpha * pv[c];
      R rv = rv0[c] - alpha * av[c];
      R zv = rv / dv[c];
      r[j] = rv; z[j] = zv;
      rz += (double)rv * (double)zv;
      rr += (double)rv * (double)rv;
    }
  }
  double v[2] = {rz, rr}, t[2], sum[2];
  block_sum_n<2>(v, sh, t);
  if (grid_reduce<2>(t, part, ctr, sh, sum)) {
    const double rz_new = sum[0], rrs = sum[1];
    if (threadIdx.x == 0) {
      s->beta = rz_new / s->rz;
      s->rz = rz_new;
      s->rr = rrs;
      s->iters += 1;
      if (rrs <= s->tol2 || s->iters >= s->maxit || !(rrs == rrs)) s->done = 1;
    }
  }
}

// ---- CFL-limited time step ------------------------------------------------------------
// The fastest particle speed and the smallest density of a particle set, as the bit
// patterns of non-negative doubles (whose unsigned order is their numeric order), so an
// integer max / min gives the same result in any order.  out[0]: max |v_p|^2 (start 0),
// out[1]: min m_p / V0_p (start +inf).  |v|^2 = (v0^2 + v1^2) + v2^2 with separate
// roundings, as any reference summing axis by axis in FP64.
MPM_DEV double speed2_rn(const double* v, int D) {
  double s = mul_nc(v[0], v[0]);
  for (int a = 1; a < D; ++a) s = add_nc(s, mul_nc(v[a], v[a]));
  return s;
}

__global__ void k_cfl_init(unsigned long long* out) {
  out[0] = 0ull;
  out[1] = 0x7FF0000000000000ull;   // +inf
}

template <int D, typename R>
__global__ void k_max_speed(int n, const R* v, const R* m, const R* V0, unsigned long long* out) {
  double vmax2 = 0, rmin = __longlong_as_double(0x7FF0000000000000ll);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    double vv[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) vv[a] = (double)v[(size_t)a * n + p];
    vmax2 = fmax(vmax2, speed2_rn(vv, D));
    rmin = fmin(rmin, (double)m[p] / (double)V0[p]);
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    vmax2 = fmax(vmax2, __shfl_xor(vmax2, o, kWave));
    rmin = fmin(rmin, __shfl_xor(rmin, o, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(vmax2));
    atomicMin(&out[1], (unsigned long long)__double_as_longlong(rmin));
  }
}

// ---- collision objects -------------------------------------------------------------------
// Static half-spaces (x - o) . n < 0 with Coulomb friction, applied to v^ at the nodes of
// the active tiles after the momentum update, object by object.  The inside test is taken
// in FP64 with products and sums in axis order (the oracle's arithmetic); the velocity
// update in the arithmetic of R.
struct Planes {
  int n;
  double o[4][3], nrm[4][3], mu[4];
};

template <int D, typename R>
__global__ void k_collide(const int* tile_list, int nelem, int nn, int nt, double dx, Planes pl, R* v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nelem) return;
  const int tile = tile_list[e >> 6];
  const int node = tile * kTileNodes + (e & 63);
  int i[3] = {0, 0, 0};
  tiled_coords<D>(tile, e & 63, nt, i);
  R vv[D];
#pragma unroll
  for (int a = 0; a < D; ++a) vv[a] = v[(int64_t)a * nn + node];
  for (int k = 0; k < pl.n; ++k) {
    double phi = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) phi = add_nc(phi, mul_nc(sub_nc(mul_nc((double)i[a] + 0.5, dx), pl.o[k][a]), pl.nrm[k][a]));
    if (phi > 0) continue;
    R vn = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) vn += vv[a] * (R)pl.nrm[k][a];
    if (!(vn < 0)) continue;
    R vt[D], t2 = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      vt[a] = vv[a] - vn * (R)pl.nrm[k][a];
      t2 += vt[a] * vt[a];
    }
    const R tl = sqrt(t2);
    const R keep = fmax(R(0), tl + (R)pl.mu[k] * vn);
    const R sc = tl > 0 ? keep / tl : R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) vv[a] = vt[a] * sc;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) v[(int64_t)a * nn + node] = vv[a];
}

// ---- preconditioned MINRES (Paige and Saunders 1975) -----------------------------------
// For the Newton system with the exact surface Hessian, which may be indefinite.  The
// Lanczos process on the Jacobi-preconditioned operator gives a tridiagonal matrix; one
// Givens rotation per iteration keeps its QR factor, and the iterate moves along the
// directions w of that factor, so the preconditioned residual norm phibar never grows.
// Scalars in FP64 on the device; every kernel of an iteration returns at once when the
// solve has finished.  Vectors: y (preconditioned residual, the Hessian's input), t (the
// Hessian's output, then the next residual), v (Lanczos vector), r_prev, r_cur, w, w_prev,
// x.
struct MinresScal {
  double beta, beta_prev, alpha, dbar, eps, eps_prev, delta, phibar, phi, c, s, gamma, tol;
  int done, iters, maxit, breakdown;
};

// r_prev = r_cur = bscale b, y = r / diag, x = w = w_prev = 0; beta = sqrt(r . y).
template <typename R>
__global__ void k_minres_start(const int* tl, int nelem, int nn, int ncomp, const R* b, R bscale, const R* diag,
                               R* x, R* rprev, R* rcur, R* y, R* w, R* wprev, double* part, unsigned* ctr,
                               MinresScal* ms, double rel_tol, int maxit) {
  __shared__ double sh[kRedSh];
  double ry = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    const int node = elem_node(tl, e);
    R bv[kMaxComp], dv[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      bv[c] = b[c * nn + node];
      dv[c] = diag[c * nn + node];
    }
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      const R rv = bscale * bv[c], yv = rv / dv[c];
      x[j] = 0; w[j] = 0; wprev[j] = 0;
      rprev[j] = rv; rcur[j] = rv; y[j] = yv;
      ry += (double)rv * (double)yv;
    }
  }
  double t = block_sum(ry, sh), r;
  if (grid_reduce<1>(&t, part, ctr, sh, &r) && threadIdx.x == 0) {
    const double beta = sqrt(r > 0 ? r : 0.0);
    ms->beta = beta; ms->beta_prev = 0; ms->alpha = 0; ms->dbar = 0; ms->eps = 0; ms->eps_prev = 0;
    ms->delta = 0; ms->phibar = beta; ms->phi = 0; ms->c = -1; ms->s = 0; ms->gamma = 0;
    ms->tol = rel_tol * beta;
    ms->iters = 0; ms->maxit = maxit; ms->breakdown = 0;
    ms->done = (beta == 0.0 || !(beta == beta) || maxit <= 0) ? 1 : 0;
  }
}

// Lanczos, first half (t holds A y): v = y / beta, t = A v - (beta / beta_prev) r_prev
// (no r_prev term on the first iteration), alpha = v . t.
template <typename R>
__global__ void k_minres_lanczos(const int* tl, int nelem, int nn, int ncomp, const R* y, R* t, R* v, const R* rprev,
                                 double* part, unsigned* ctr, MinresScal* ms) {
  __shared__ double sh[kRedSh];
  if (ms->done) return;
  const double beta = ms->beta;
  const R inv = (R)(1.0 / beta), co = ms->iters > 0 ? (R)(beta / ms->beta_prev) : R(0);
  double va = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    const int node = elem_node(tl, e);
    R yv[kMaxComp], tv[kMaxComp], rv[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      yv[c] = y[j]; tv[c] = t[j]; rv[c] = rprev[j];
    }
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      const R vv = yv[c] * inv, tn = tv[c] * inv - co * rv[c];
      v[j] = vv; t[j] = tn;
      va += (double)vv * (double)tn;
    }
  }
  double bsum = block_sum(va, sh), a;
  if (grid_reduce<1>(&bsum, part, ctr, sh, &a) && threadIdx.x == 0) ms->alpha = a;
}

// Lanczos, second half, and the rotation: t -= (alpha / beta) r_cur (t becomes the next
// residual), y = t / diag, beta' = sqrt(t . y); then the previous rotation applied to the
// new column and the rotation that annihilates beta'.  Sets done at phibar <= tol or at
// the iteration cap.
template <typename R>
__global__ void k_minres_rotate(const int* tl, int nelem, int nn, int ncomp, R* t, const R* rcur, const R* diag,
                                R* y, double* part, unsigned* ctr, MinresScal* ms) {
  __shared__ double sh[kRedSh];
  if (ms->done) return;
  const R co = (R)(ms->alpha / ms->beta);
  double ty = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    const int node = elem_node(tl, e);
    R tv[kMaxComp], rv[kMaxComp], dv[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      tv[c] = t[j]; rv[c] = rcur[j]; dv[c] = diag[j];
    }
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      const R tn = tv[c] - co * rv[c], yn = tn / dv[c];
      t[j] = tn; y[j] = yn;
      ty += (double)tn * (double)yn;
    }
  }
  double bsum = block_sum(ty, sh), b2;
  if (grid_reduce<1>(&bsum, part, ctr, sh, &b2) && threadIdx.x == 0) {
    const double beta = sqrt(b2 > 0 ? b2 : 0.0), alpha = ms->alpha;
    ms->beta_prev = ms->beta;
    ms->beta = beta;
    ms->eps_prev = ms->eps;
    ms->delta = ms->c * ms->dbar + ms->s * alpha;
    const double gbar = ms->s * ms->dbar - ms->c * alpha;
    ms->eps = ms->s * beta;
    ms->dbar = -ms->c * beta;
    const double gamma = fmax(hypot(gbar, beta), 2.220446049250313e-16);
    ms->gamma = gamma;
    ms->c = gbar / gamma;
    ms->s = beta / gamma;
    ms->phi = ms->c * ms->phibar;
    ms->phibar = ms->s * ms->phibar;
    ms->iters += 1;
    if (!(b2 == b2) || !(alpha == alpha)) ms->breakdown = 1;
    if (ms->breakdown || fabs(ms->phibar) <= ms->tol || ms->iters >= ms->maxit || beta == 0.0) ms->done = 1;
  }
}

// The iterate of iteration `it` (skipped unless that iteration's rotation ran): w' = (v -
// eps_prev w_prev - delta w) / gamma, written over w_prev, x += phi w'.
template <typename R>
__global__ void k_minres_step(const int* tl, int nelem, int nn, int ncomp, const R* v, const R* w, R* wprev, R* x,
                              const MinresScal* ms, int it) {
  if (ms->iters != it) return;
  const R ep = (R)ms->eps_prev, de = (R)ms->delta, ig = (R)(1.0 / ms->gamma), ph = (R)ms->phi;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    const int node = elem_node(tl, e);
    R vv[kMaxComp], wv[kMaxComp], pv[kMaxComp], xv[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      vv[c] = v[j]; wv[c] = w[j]; pv[c] = wprev[j]; xv[c] = x[j];
    }
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= ncomp) break;
      const int j = c * nn + node;
      const R wn = (vv[c] - ep * pv[c] - de * wv[c]) * ig;
      wprev[j] = wn;
      x[j] = xv[c] + ph * wn;
    }
  }
}

// After the loop: breakdown at the first iteration takes the preconditioned residual.
template <typename R>
__global__ void k_cg_fixup(const int* tl, int nelem, int nn, int ncomp, const CgScal* s, R* x, const R* z) {
  if (!(s->breakdown && s->iters == 0)) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    for (int c = 0; c < ncomp; ++c) x[c * nn + node] = z[c * nn + node];
  }
}

// y = a + s b on free components (s from a device double or a host value).
template <typename R>
__global__ void k_axpy_to(const int* tl, int nelem, int nn, int ncomp, const R* a, const R* b, double sh,
                          R* y) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    R av[kMaxComp], bv[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
      if (c < ncomp) { av[c] = a[c * nn + node]; bv[c] = b[c * nn + node]; }
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
      if (c < ncomp) y[c * nn + node] = av[c] + (R)sh * bv[c];
  }
}

// v^ = P v^n.
template <typename R>
__global__ void k_project_copy(const int* tl, int nelem, int nn, int ncomp, const uint8_t* fr, const R* a,
                               R* y) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    uint8_t f = fr[node];
    R av[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
      if (c < ncomp) av[c] = a[c * nn + node];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
      if (c < ncomp) y[c * nn + node] = ((f >> c) & 1) ? av[c] : R(0);
  }
}

template <typename R>
__global__ void k_neg(const int* tl, int nelem, int nn, int ncomp, const R* a, R* y) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    for (int c = 0; c < ncomp; ++c) y[c * nn + node] = -a[c * nn + node];
  }
}

// Momentum sums over nodes with mass: slots 0..D-1 sum m (v^ - v^n), slot D sum m,
// slots D+1..2D sum m v^; the last block writes them to dst[0..2D].
template <int D, typename R>
__global__ void k_mom_sums(const int* tl, int nelem, int nn, const uint8_t* fr, const R* m, const R* vh,
                           const R* vn, double* part, unsigned* ctr, double* dst) {
  __shared__ double sh[(2 * D + 1) * kNodeThreads];
  double s[2 * D + 1];
  for (int k = 0; k < 2 * D + 1; ++k) s[k] = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    if (!(fr[node] & 0x80)) continue;
    double mm = m[node];
    s[D] += mm;
    for (int a = 0; a < D; ++a) {
      s[a] += mm * ((double)vh[a * nn + node] - (double)vn[a * nn + node]);
      s[D + 1 + a] += mm * (double)vh[a * nn + node];
    }
  }
  double t[2 * D + 1], r[2 * D + 1];
  block_sum_n<2 * D + 1>(s, sh, t);
  if (grid_reduce<2 * D + 1>(t, part, ctr, sh, r) && threadIdx.x == 0)
    for (int k = 0; k < 2 * D + 1; ++k) dst[k] = r[k];
}

// The start of the next Newton iteration's CG, fused into the translation correction of
// the trial that precedes it: r = -g at the corrected trial point, z = r / diag, p = z,
// x = 0 (the start of a CG for the right side -g, as k_cg_start forms it), and its
// scalars with the tolerance of the device's Newton decision, marked done when the
// iteration does not follow.  x == nullptr: none.
template <typename R>
struct NextCgStart {
  R* x;
  R* r;
  R* z;
  R* p;
  const R* diag;
  CgScal* cs;
  int maxit;
};

// Exact minimization of Phi along rigid translations: v^ -= c on nodes with mass,
// c_a = [sum m (v^ - v^n) - dt g_a sum m] / sum m.  e and D are translation invariant, so
// the projected gradient moves by exactly -m c; the grid sum of |grad|^2 after the move
// goes to *gn2.  skip (a constrained component; uniform in the grid): no correction, and
// *gn2 keeps the merge's sum.  Also forms, in the same pass and with the same per-node
// arithmetic and summation order as k_mom_sums, the momentum sums of the (corrected)
// point into mom[0..2D], and the next CG's start (nx) after the Newton decision (nd).
template <int D, typename R>
__global__ void k_mom_fix(const int* tl, int nelem, int nn, const uint8_t* fr, const R* m, const double* red,
                          double dt, double g0, double g1, double g2, R* vh, R* grad, double* part, unsigned* ctr,
                          double* gn2, const int* skip, const R* vn, double* mom, NextCgStart<R> nx,
                          NewtonDecide nd) {
  constexpr int NV = 2 * D + 4;   // |g|^2, r.z, r.r, momentum sums
  __shared__ double sh[NV * kNodeThreads];
  const bool fix = !*skip;
  double msum = red[D];
  double gg[3] = {g0, g1, g2};
  R c[D];
  for (int a = 0; a < D; ++a) c[a] = fix ? (R)((red[a] - dt * gg[a] * msum) / msum) : R(0);
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    // every load of the node first: the stores below may alias them for the compiler
    const uint8_t f = fr[node];
    const bool dof = f & 0x80;
    const R mn = m[node];
    R vv[D], gv[D], vnv[D], dg[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int j = a * nn + node;
      gv[a] = grad[j];
      vv[a] = vh[j];
      vnv[a] = vn[j];
      dg[a] = nx.x ? nx.diag[j] : R(1);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int j = a * nn + node;
      if (fix && dof) {
        vv[a] -= c[a];
        vh[j] = vv[a];
        gv[a] -= mn * c[a];
        grad[j] = gv[a];
      }
      v[0] += (double)gv[a] * (double)gv[a];
      if (nx.x) {
        R rv = R(-1) * gv[a];
        R zv = rv / dg[a];
        nx.x[j] = 0;
        nx.r[j] = rv; nx.z[j] = zv; nx.p[j] = zv;
        v[1] += (double)rv * (double)zv;
        v[2] += (double)rv * (double)rv;
      }
    }
    if (dof) {
      double mm = mn;
      v[3 + D] += mm;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        v[3 + a] += mm * ((double)vv[a] - (double)vnv[a]);
        v[3 + D + 1 + a] += mm * (double)vv[a];
      }
    }
  }
  double t[NV], r[NV];
  block_sum_n<NV>(v, sh, t);
  if (grid_reduce<NV>(t, part, ctr, sh, r) && threadIdx.x == 0) {
    if (fix) *gn2 = r[0];
    for (int k = 0; k < 2 * D + 1; ++k) mom[k] = r[3 + k];
    if (nx.x) {
      const bool go = nd.scal ? newton_decide(nd) : true;
      cg_init(nx.cs, r[1], r[2], nd.scal ? nd.scal[nd.tol_slot] : 0.0, nx.maxit);
      if (!go) nx.cs->done = 1;
    }
  }
}

// Explicit update (q^ = 0): v^ = P[v^n - f/m + dt g] with f = dPsi/dv^ evaluated by the
// caller (J and surface terms at v^ = 0, viscosity at v^n).
template <int D, typename R>
__global__ void k_explicit_update(const int* tl, int nelem, int nn, const uint8_t* fr, const R* m, const R* vn,
                                  const R* f, R g0, R g1, R g2, R dt, R* vh) {
  R gg[3] = {g0, g1, g2};
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    int node = elem_node(tl, e);
    uint8_t fl = fr[node];
    for (int a = 0; a < D; ++a) {
      int j = a * nn + node;
      vh[j] = ((fl >> a) & 1) ? vn[j] - f[j] / m[node] + dt * gg[a] : R(0);
    }
  }
}

// Counts the degrees of freedom (nodes with mass) into misc[2] and sets misc[1] when any
// node with mass has a constrained component.  Grid-stride over the active nodes with one
// atomic pair per block (same-address atomics serialize across the grid).
template <int D>
__global__ void k_dof_flags(const int* tl, int nelem, const uint8_t* fr, int* misc) {
  int cnt = 0, con = 0;
  const uint8_t all = (uint8_t)((1u << D) - 1);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nelem; e += gridDim.x * blockDim.x) {
    uint8_t f = fr[elem_node(tl, e)];
    if (f & 0x80) {
      cnt += 1;
      con |= (f & all) != all;
    }
  }
  __shared__ int scnt, scon;
  if (threadIdx.x == 0) { scnt = 0; scon = 0; }
  __syncthreads();
  if (cnt) atomicAdd(&scnt, cnt);
  if (con) atomicOr(&scon, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (scnt) atomicAdd(&misc[2], scnt);
    if (scon) atomicOr(&misc[1], 1);
  }
}

}  // namespace mpm
