// Shared device helpers of the MPM hot path: node/cell tiling, the quadratic B-spline in
// cell-relative form, wave-shuffle reductions and the status word.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpm.h"

#define MPM_DEV __device__ __forceinline__
#define MPM_HD __host__ __device__ __forceinline__

namespace mpm {

// Double products, sums and differences rounded one at a time.  HIP contracts a product
// and a sum into one fused multiply-add by default (so do the _rn intrinsics, which are
// plain operators here); under this pragma the operations carry no contraction flag, so
// they round exactly as a host computation written in the same order.
MPM_DEV double mul_nc(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
MPM_DEV double add_nc(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}
MPM_DEV double sub_nc(double a, double b) {
#pragma clang fp contract(off)
  return a - b;
}

constexpr int kTileNodes = 64;   // nodes per tile: 4x4x4 (3D) or 8x8 (2D)
constexpr int kMaxPartials = 1024;
constexpr int kWave = 64;

template <int D> struct Tiling;
template <> struct Tiling<3> { static constexpr int E = 4; static constexpr int LOG = 2; };
template <> struct Tiling<2> { static constexpr int E = 8; static constexpr int LOG = 3; };

// Index of node / cell (i0,i1,i2) in tile-major order (include/mpm.h, mpm_node_index).
template <int D>
MPM_HD int64_t tiled_index(const int* i, int nt) {
  constexpr int E = Tiling<D>::E, L = Tiling<D>::LOG;
  int64_t tile = (i[0] >> L) + (int64_t)nt * ((i[1] >> L) + (D == 3 ? (int64_t)nt * (i[2] >> L) : 0));
  int local = (i[0] & (E - 1)) + E * ((i[1] & (E - 1)) + (D == 3 ? E * (i[2] & (E - 1)) : 0));
  return tile * kTileNodes + local;
}

// Multi-index of node number tile*64+local.
template <int D>
MPM_HD void tiled_coords(int64_t tile, int local, int nt, int* i) {
  constexpr int E = Tiling<D>::E, L = Tiling<D>::LOG;
  int64_t t0 = tile % nt;
  int64_t rest = tile / nt;
  i[0] = (int)(t0 << L) + (local & (E - 1));
  if (D == 3) {
    int64_t t1 = rest % nt, t2 = rest / nt;
    i[1] = (int)(t1 << L) + ((local >> L) & (E - 1));
    i[2] = (int)(t2 << L) + (local >> (2 * L));
  } else {
    i[1] = (int)(rest << L) + (local >> L);
  }
}

// Quadratic B-spline at cell-centred nodes, in the cell-relative variable f = x/dx - c,
// c = floor(x/dx), f in [0,1).  The point's 3^D stencil is nodes c-1+k, k = 0,1,2, with
// 1D weights  k=0: (1-f)^2/2,  k=1: 3/4 - (f-1/2)^2,  k=2: f^2/2
// and derivatives (per dx)  -(1-f),  1-2f,  f.  (Same kernel as N(u) of Section 4.2 with
// u = f + 1/2 - k.)
template <typename R>
MPM_DEV R bs_w(int k, R f) {
  return k == 0 ? R(0.5) * (R(1) - f) * (R(1) - f)
       : (k == 1 ? R(0.75) - (f - R(0.5)) * (f - R(0.5)) : R(0.5) * f * f);
}
template <typename R>
MPM_DEV R bs_dw(int k, R f) {
  return k == 0 ? f - R(1) : (k == 1 ? R(1) - R(2) * f : f);
}

template <int D, typename R>
struct Stencil {
  int c[D];        // cell of the point
  R f[D];          // cell-relative position
  R w[D][3];       // 1D weights of nodes c-1+k
  R dw[D][3];      // 1D derivatives, already divided by dx
};

// Cell and cell-relative coordinate of a position.  Positions outside [dx, 1-dx) are
// clamped (so every access stays inside the grid) and reported through *bad.
template <int D, typename R>
MPM_DEV void locate(const R* x, int n, R fn, int* c, R* f, bool* bad) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    R xs = x[a] * fn;
    R cf = floor(xs);
    bool ok = (xs >= R(1)) && (xs < R(n - 1));   // also false for NaN
    if (!ok) { *bad = true; cf = xs < R(1) || !(xs == xs) ? R(1) : R(n - 2); xs = cf; }
    c[a] = (int)cf;
    f[a] = xs - cf;
  }
}

template <int D, typename R>
MPM_DEV void make_stencil(const R* x, int n, R fn, Stencil<D, R>& s, bool* bad) {
  locate<D, R>(x, n, fn, s.c, s.f, bad);
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.w[a][k] = bs_w<R>(k, s.f[a]);
      s.dw[a][k] = bs_dw<R>(k, s.f[a]) * fn;
    }
  }
}

// Loop over the 3^D stencil offsets, k0 fastest.
template <int D, class F>
MPM_DEV void for_stencil(F&& fn) {
  if constexpr (D == 3) {
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2)
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1)
#pragma unroll
        for (int k0 = 0; k0 < 3; ++k0) fn(k0, k1, k2);
  } else {
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1)
#pragma unroll
      for (int k0 = 0; k0 < 3; ++k0) fn(k0, k1, 0);
  }
}

// Weight and gradient of stencil node (k0,k1,k2).
template <int D, typename R>
MPM_DEV R node_weight(const Stencil<D, R>& s, int k0, int k1, int k2, R* g) {
  if constexpr (D == 3) {
    R wx = s.w[0][k0], wy = s.w[1][k1], wz = s.w[2][k2];
    g[0] = s.dw[0][k0] * wy * wz;
    g[1] = wx * s.dw[1][k1] * wz;
    g[2] = wx * wy * s.dw[2][k2];
    return wx * wy * wz;
  } else {
    R wx = s.w[0][k0], wy = s.w[1][k1];
    g[0] = s.dw[0][k0] * wy;
    g[1] = wx * s.dw[1][k1];
    return wx * wy;
  }
}

// Weight and gradient of node i for a point in cell c with cell-relative f (node-gather
// form: k_a = i_a - c_a + 1 in {0,1,2}).
template <int D, typename R>
MPM_DEV R weight_from_cell(const int* k, const R* f, R fn, R* g) {
  R w[D], dw[D];
#pragma unroll
  for (int a = 0; a < D; ++a) { w[a] = bs_w<R>(k[a], f[a]); dw[a] = bs_dw<R>(k[a], f[a]) * fn; }
  if constexpr (D == 3) {
    g[0] = dw[0] * w[1] * w[2];
    g[1] = w[0] * dw[1] * w[2];
    g[2] = w[0] * w[1] * dw[2];
    return w[0] * w[1] * w[2];
  } else {
    g[0] = dw[0] * w[1];
    g[1] = w[0] * dw[1];
    return w[0] * w[1];
  }
}

// Fused multiply-add, one rounding.
MPM_DEV float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
MPM_DEV double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---- deterministic reductions -------------------------------------------------------
MPM_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}

// Sum over the block (fixed order: lanes by shuffle tree, then waves in index order).
// Result valid in thread 0.  sh must hold blockDim/64 doubles.
MPM_DEV double block_sum(double v, double* sh) {
  v = wave_sum(v);
  int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) {
    int nw = (blockDim.x + kWave - 1) / kWave;
    for (int k = 0; k < nw; ++k) r += sh[k];
  }
  return r;
}

// ---- deterministic grid reduction without a second launch ----------------------------
// Thread 0 of every block publishes its NV partials with device-scope stores (written
// through to the level shared by all XCDs), waits until they are acknowledged and takes a
// ticket of its group of kRedGroup blocks.  The last block of a group sums the group's
// partials in index order, publishes the group sum and takes a ticket of the grid; the
// last group sums the group sums in index order.  The result therefore does not depend
// on which blocks finish first.  Same-address atomics serialize (tens of ns each across
// XCDs), so two levels keep the serial chain at kRedGroup + groups tickets instead of one
// per block; the counters sit on separate 128-byte lines.  No cache writeback or
// invalidate is issued.  Counters return to zero for the next use.
//   part: partial v of block b at part[v * kRedSlot + b], group sums at kRedGroupOff + g;
//   ctr:  kCtrSite unsigned counters of this reduction site.
constexpr int kRedSlot = 1 << 18;
constexpr int kRedGroup = 64;
constexpr int kRedGroupOff = 1 << 17;                  // max blocks of a reducing grid
constexpr int kMaxRedGroups = kRedGroupOff / kRedGroup;
constexpr int kCtrStride = 32;
constexpr int kCtrSite = (1 + kMaxRedGroups) * kCtrStride;
constexpr int kRedSh = 64;   // LDS doubles of a block that reduces single values (grid_reduce needs NV <= kRedSh)

MPM_DEV void publish(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

MPM_DEV unsigned take_ticket(unsigned* c) {
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's published stores are acknowledged
  return __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

MPM_DEV void reset_ticket(unsigned* c) { __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Sum of part[0..nb) in fixed order by one block (result in thread 0); device-scope loads
// see every block's published partial.
MPM_DEV double block_sum_array(const double* part, int nb, double* sh) {
  constexpr int U = 8;   // loads in flight per thread
  double v = 0;
  for (int k0 = threadIdx.x; k0 < nb; k0 += U * blockDim.x) {
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int k = k0 + u * blockDim.x;
      t[u] = k < nb ? __hip_atomic_load(part + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v += t[u];
  }
  return block_sum(v, sh);
}

// Lanes that sum one value in the transposed block sums below: the largest power of two
// up to a wave with nv * L <= nt.
MPM_DEV int red_lanes(int nv, int nt) {
  int l = kWave;
  while (l > 1 && nv * l > nt) l >>= 1;
  return l;
}

// Shuffle tree over aligned groups of L lanes (L a power of two dividing the wave): the
// first lane of each group gets the group's sum.  Every lane of the wave takes part.
MPM_DEV double group_sum(double p, int L) {
  for (int o = L / 2; o > 0; o >>= 1) p += __shfl_down(p, o, kWave);
  return p;
}

// NV block sums at once (each thread's v[k]; results in thread 0's out[k]), transposed:
// the values go to LDS (sh must hold NV * blockDim doubles), and value k is summed by the
// L = red_lanes(NV, blockDim) lanes k L .. k L + L - 1, lane q over the entries q, q + L,
// ... in index order, then by a shuffle tree over the L lanes.  The order is fixed.  All
// values share one tree of log2(L) steps (one tree per value serializes on the LDS
// counter).
template <int NV>
MPM_DEV void block_sum_n(const double* v, double* sh, double* out) {
  const int nt = blockDim.x, t = threadIdx.x;
  const int L = red_lanes(NV, nt);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) sh[k * nt + t] = v[k];
  __syncthreads();
  const int k = t / L, q = t % L;
  double p = 0;
  if (k < NV)
    for (int i = q; i < nt; i += L) p += sh[k * nt + i];
  p = group_sum(p, L);
  __syncthreads();
  if (k < NV && q == 0) sh[k] = p;
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) out[j] = sh[j];
  }
}

// Sums of NV published arrays part[v * kRedSlot + (0..nb)] in fixed order (thread 0's
// out), transposed as in block_sum_n, straight from the device-scope loads (sh must hold
// NV doubles).
template <int NV>
MPM_DEV void block_sum_arrays(const double* part, int nb, double* sh, double* out) {
  constexpr int U = 4;   // loads in flight per lane
  const int t = threadIdx.x, L = red_lanes(NV, blockDim.x);
  const int k = t / L, q = t % L;
  double p = 0;
  if (k < NV) {
    const double* src = part + (size_t)k * kRedSlot;
    for (int i0 = q; i0 < nb; i0 += U * L) {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * L;
        x[u] = i < nb ? __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) p += x[u];
    }
  }
  p = group_sum(p, L);
  __syncthreads();
  if (k < NV && q == 0) sh[k] = p;
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) out[j] = sh[j];
  }
}

// vals: the block's NV sums (read in thread 0).  Returns true in the one block that holds
// the grid sums, in out[0..NV) of thread 0.  Every thread of every block must call it.
template <int NV>
MPM_DEV bool grid_reduce(const double* vals, double* part, unsigned* ctr, double* sh, double* out) {
  __shared__ int flag;
  const int b = blockIdx.x, nb = gridDim.x;
  const int g = b / kRedGroup, ng = (nb + kRedGroup - 1) / kRedGroup;
  const int gsz = min(kRedGroup, nb - g * kRedGroup);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) publish(part + (size_t)v * kRedSlot + b, vals[v]);
    unsigned* gc = ctr + (size_t)(1 + g) * kCtrStride;
    bool last = take_ticket(gc) == (unsigned)(gsz - 1);
    if (last) reset_ticket(gc);
    flag = last;
  }
  __syncthreads();
  if (!flag) return false;
  double gs[NV];
  block_sum_arrays<NV>(part + (size_t)g * kRedGroup, gsz, sh, gs);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) publish(part + (size_t)v * kRedSlot + kRedGroupOff + g, gs[v]);
    bool last = take_ticket(ctr) == (unsigned)(ng - 1);
    if (last) reset_ticket(ctr);
    flag = last;
  }
  __syncthreads();
  if (!flag) return false;
  block_sum_arrays<NV>(part + kRedGroupOff, ng, sh, out);
  return true;
}

// Latched device status word bits.
// ST_STALL: a bounded device-side wait gave up; ST_INTERNAL: a consistency check failed
// (results of the step are invalid in both cases).
enum : int { ST_DOMAIN = 1, ST_NONFINITE = 2, ST_NOCONV = 4, ST_STALL = 8, ST_INTERNAL = 16 };

MPM_DEV void flag_status(int* st, int bit) { atomicOr(st, bit); }

}  // namespace mpm
