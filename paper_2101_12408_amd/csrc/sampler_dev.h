// Surface samples on the device (Section 4.1.1): the union-of-spheres level set around the
// particles, its zero isocontour by marching tetrahedra (3D, six tets around each cube's
// main diagonal) or marching triangles (2D, two per square), and per-element uniform
// samples with area-weighted outward normals.
//
// The samples are the host input stage's (mpm_sample_surface) bit for bit: the same
// element ids (cube c = i0 + (n-1)(i1 + (n-1) i2), id = (c T + t) 2 + j), the same
// SplitMix64 counter draws keyed by (seed, step, id), and every floating-point operation
// of the geometry in the same order with single roundings (mul_nc / add_nc / sub_nc keep
// the compiler from contracting a product and a sum into one fused operation; division
// and square root are correctly rounded).
//
// Passes (dense over nodes and cubes, natural order):
//   k_smp_keys / sort      particles binned by cell (floor(x / dx), clamped)
//   k_smp_gather           positions in cell order
//   k_smp_inside           flag bit 1: a particle closer than r (its 2^d node box)
//   k_smp_need             flag bit 2: the node has an inside node within one node
//   k_smp_phi              phi = exact nearest distance - r at the flagged nodes,
//                          searched ring by ring over the binned cells
//   k_smp_count            per cube with an inside corner: its elements' sample counts
//   scan                   sample offsets per cube (element id order)
//   k_smp_emit             the samples, s and dA as [dim][total], label [total]
#pragma once

#include "kernels.h"

namespace mpm {

constexpr uint64_t kSmpGolden = 0x9E3779B97F4A7C15ull;

MPM_DEV uint64_t smp_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Draw j of element e's stream under key, uniform in [0, 1) with 53 bits.
MPM_DEV double smp_draw(uint64_t key, uint64_t e, uint64_t j) {
  const uint64_t s = smp_mix(key + (e + 1) * kSmpGolden);
  const uint64_t z = smp_mix(s + (j + 1) * kSmpGolden);
  return (double)(z >> 11) * 0x1p-53;
}

struct SmpArgs {
  int n, nt;
  double dx, r, rho;
  uint64_t key;
  int has_label;
  double lo[3], hi[3];
};

MPM_DEV int64_t smp_node(const int* i, int n, int D) {
  return i[0] + (int64_t)n * (i[1] + (D == 3 ? (int64_t)n * i[2] : 0));
}

template <int D>
MPM_DEV void smp_cell(const double* x, int n, double dx, int* c) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double v = floor(x[a] / dx);
    v = fmin(fmax(v, 0.0), (double)(n - 1));
    c[a] = (int)v;
  }
}

// Cell key (the step's tiled cell numbering) and count of every particle.
template <int D, typename R>
__global__ void k_smp_keys(const R* pos, int cnt, int n, int nt, double dx, int* key, int* ccount) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < cnt;
  int k = 0;
  if (act) {
    double x[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = (double)pos[(int64_t)a * cnt + i];
    int c[D];
    smp_cell<D>(x, n, dx, c);
    k = (int)tiled_index<D>(c, nt);
    key[i] = k;
  }
  int head, len;
  wave_run(k, act, head, len);
  if (act && __lane_id() == head) atomicAdd(&ccount[k], len);
}

template <int D, typename R>
__global__ void k_smp_gather(const R* pos, int cnt, const int* perm, R* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cnt) return;
  const int p = perm[k];
#pragma unroll
  for (int a = 0; a < D; ++a) out[(int64_t)a * cnt + k] = pos[(int64_t)a * cnt + p];
}

// Bit 1 of flag[node]: some particle closer than r.  r < dx, so such nodes lie in the 2^d
// box of nodes around the particle.  Every writer stores the same byte value.
template <int D, typename R>
__global__ void k_smp_inside(const R* pos, int cnt, SmpArgs a, uint8_t* flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= cnt) return;
  double x[D];
  int base[D];
#pragma unroll
  for (int q = 0; q < D; ++q) {
    x[q] = (double)pos[(int64_t)q * cnt + p];
    base[q] = (int)floor(sub_nc(x[q] / a.dx, 0.5));
  }
  for (int b = 0; b < (1 << D); ++b) {
    int i[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      i[q] = base[q] + ((b >> q) & 1);
      ok = ok && i[q] >= 0 && i[q] < a.n;
    }
    if (!ok) continue;
    double d2 = 0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const double t = sub_nc(mul_nc((double)i[q] + 0.5, a.dx), x[q]);
      d2 = add_nc(d2, mul_nc(t, t));
    }
    if (sub_nc(sqrt(d2), a.r) < 0) flag[smp_node(i, a.n, D)] = 1;
  }
}

// Bit 2: an inside node within one node in every axis (every corner of a cube that has an
// inside corner is such a node).  Each thread writes only its own byte.
template <int D>
__global__ void k_smp_need(uint8_t* flag, int n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nn = (int64_t)n * n * (D == 3 ? n : 1);
  if (k >= nn) return;
  const int i[3] = {(int)(k % n), (int)((k / n) % n), D == 3 ? (int)(k / ((int64_t)n * n)) : 0};
  bool near = false;
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dxo = -1; dxo <= 1; ++dxo) {
        const int j[3] = {i[0] + dxo, i[1] + dy, i[2] + dz};
        bool ok = true;
#pragma unroll
        for (int q = 0; q < D; ++q) ok = ok && j[q] >= 0 && j[q] < n;
        if (ok && (flag[smp_node(j, n, D)] & 1)) near = true;
      }
  if (near) flag[k] = flag[k] | 2;
}

// phi at the nodes with bit 2: the nearest particle over the cells within three cells,
// searched in shells of growing Chebyshev radius R; every particle outside the shells
// searched so far is at least (R + 1/2) dx away (the node is its cell's centre), so the
// search stops once the best distance is within that bound.
template <int D, typename R>
__global__ void k_smp_phi(const R* xs, int cnt, const int* start, SmpArgs a, const uint8_t* flag, double* phi) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = a.n;
  int64_t nn = (int64_t)n * n * (D == 3 ? n : 1);
  if (k >= nn || !(flag[k] & 2)) return;
  const int i[3] = {(int)(k % n), (int)((k / n) % n), D == 3 ? (int)(k / ((int64_t)n * n)) : 0};
  double pos[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < D; ++q) pos[q] = mul_nc((double)i[q] + 0.5, a.dx);
  double best = 1e300;
  for (int Rg = 0; Rg <= 3; ++Rg) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < D; ++q) {
      lo[q] = max(i[q] - Rg, 0);
      hi[q] = min(i[q] + Rg, n - 1);
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          const int c[3] = {x, y, z};
          int ring = 0;
#pragma unroll
          for (int q = 0; q < D; ++q) ring = max(ring, abs(c[q] - i[q]));
          if (ring != Rg) continue;
          const int64_t ci = tiled_index<D>(c, a.nt);
          for (int p = start[ci]; p < start[ci + 1]; ++p) {
            double d2 = 0;
#pragma unroll
            for (int q = 0; q < D; ++q) {
              const double t = sub_nc(pos[q], (double)xs[(int64_t)q * cnt + p]);
              d2 = add_nc(d2, mul_nc(t, t));
            }
            best = fmin(best, d2);
          }
        }
    const double bound = mul_nc((double)Rg + 0.5, a.dx);
    if (best <= mul_nc(bound, bound)) break;
  }
  phi[k] = sub_nc(sqrt(best), a.r);
}

// One element of the isocontour: id, vertices, orientation helper (mean of the outside
// vertices minus mean of the inside vertices of its simplex).
struct SmpElem {
  int64_t id;
  double v[3][3];
  double ori[3];
};

MPM_DEV void smp_edge(const double* xu, const double* xv, double pu, double pv, int D, double* out) {
  const double t = pu / sub_nc(pu, pv);
  for (int q = 0; q < D; ++q) out[q] = add_nc(xu[q], mul_nc(t, sub_nc(xv[q], xu[q])));
}

// Elements of simplex t of a cube (corner values cphi, positions cpos): 0, 1 or 2.
template <int D>
MPM_DEV int smp_simplex(int64_t cube, int t, const double* cphi, const double (*cpos)[3], SmpElem* e) {
  constexpr int T = D == 3 ? 6 : 2;
  constexpr int NV = D + 1;
  const int tets[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};
  const int tris[2][3] = {{0, 1, 3}, {0, 3, 2}};
  int vid[4];
  for (int k = 0; k < NV; ++k) vid[k] = D == 3 ? tets[t][k] : tris[t][k];
  double sp[4];
  bool neg[4];
  int cnt = 0, no = 0, ni = 0;
  double mo[3] = {0, 0, 0}, mi[3] = {0, 0, 0};
  for (int k = 0; k < NV; ++k) {
    sp[k] = cphi[vid[k]];
    neg[k] = sp[k] < 0;
    cnt += neg[k];
    for (int q = 0; q < D; ++q) {
      if (neg[k]) mi[q] = add_nc(mi[q], cpos[vid[k]][q]);
      else mo[q] = add_nc(mo[q], cpos[vid[k]][q]);
    }
    if (neg[k]) ++ni; else ++no;
  }
  if (cnt == 0 || cnt == NV) return 0;
  double ori[3] = {0, 0, 0};
  for (int q = 0; q < D; ++q) ori[q] = sub_nc(mo[q] / (double)no, mi[q] / (double)ni);
  const int64_t base_id = (cube * T + t) * 2;
  auto P = [&](int u, int v, double* out) { smp_edge(cpos[vid[u]], cpos[vid[v]], sp[u], sp[v], D, out); };
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < 3; ++q) e[m].ori[q] = ori[q];
  if (D == 2 || cnt == 1 || cnt == NV - 1) {
    const bool lone_in = cnt == 1;
    int a = 0;
    while (neg[a] != lone_in) ++a;
    e[0].id = base_id;
    int q = 0;
    for (int k = 0; k < NV; ++k) {
      if (k == a) continue;
      if (lone_in) P(a, k, e[0].v[q]); else P(k, a, e[0].v[q]);
      ++q;
    }
    return 1;
  }
  int ins[2], outs[2], qi = 0, qo = 0;
  for (int k = 0; k < 4; ++k) {
    if (neg[k]) ins[qi++] = k; else outs[qo++] = k;
  }
  double pac[3], pad[3], pbd[3], pbc[3];
  P(ins[0], outs[0], pac);
  P(ins[0], outs[1], pad);
  P(ins[1], outs[1], pbd);
  P(ins[1], outs[0], pbc);
  e[0].id = base_id;
  e[1].id = base_id + 1;
  for (int q = 0; q < 3; ++q) {
    e[0].v[0][q] = pac[q]; e[0].v[1][q] = pad[q]; e[0].v[2][q] = pbd[q];
    e[1].v[0][q] = pac[q]; e[1].v[1][q] = pbd[q]; e[1].v[2][q] = pbc[q];
  }
  return 2;
}

// Measure, outward unit normal and sample count of an element (count 0: degenerate, no
// samples).
template <int D>
MPM_DEV int64_t smp_measure(const SmpElem& e, const SmpArgs& a, double* nh, double* meas_out) {
  double nv[3] = {0, 0, 0}, meas;
  if (D == 3) {
    double u[3], w[3];
    for (int q = 0; q < 3; ++q) {
      u[q] = sub_nc(e.v[1][q], e.v[0][q]);
      w[q] = sub_nc(e.v[2][q], e.v[0][q]);
    }
    nv[0] = sub_nc(mul_nc(u[1], w[2]), mul_nc(u[2], w[1]));
    nv[1] = sub_nc(mul_nc(u[2], w[0]), mul_nc(u[0], w[2]));
    nv[2] = sub_nc(mul_nc(u[0], w[1]), mul_nc(u[1], w[0]));
    meas = mul_nc(0.5, sqrt(add_nc(add_nc(mul_nc(nv[0], nv[0]), mul_nc(nv[1], nv[1])),
                                               mul_nc(nv[2], nv[2]))));
  } else {
    const double ex = sub_nc(e.v[1][0], e.v[0][0]), ey = sub_nc(e.v[1][1], e.v[0][1]);
    nv[0] = -ey;
    nv[1] = ex;
    meas = sqrt(add_nc(mul_nc(ex, ex), mul_nc(ey, ey)));
  }
  *meas_out = meas;
  if (!(meas > 0)) return 0;
  const double nl = sqrt(add_nc(add_nc(mul_nc(nv[0], nv[0]), mul_nc(nv[1], nv[1])),
                                         mul_nc(nv[2], nv[2])));
  for (int q = 0; q < 3; ++q) nh[q] = nv[q] / nl;
  double dot = 0;
  for (int q = 0; q < D; ++q) dot = add_nc(dot, mul_nc(nh[q], e.ori[q]));
  if (dot < 0)
    for (int q = 0; q < 3; ++q) nh[q] = -nh[q];
  const double u0 = smp_draw(a.key, (uint64_t)e.id, 0);
  const double f = floor(add_nc(mul_nc(a.rho, meas), u0));
  return f > 1.0 ? (int64_t)f : 1;
}

// The corners of cube c: returns false when no corner is inside (bit 1), else loads phi
// and positions.
template <int D>
MPM_DEV bool smp_cube(int64_t cube, const SmpArgs& a, const uint8_t* flag, const double* phi, double* cphi,
                      double (*cpos)[3]) {
  const int m = a.n - 1;
  const int cm[3] = {(int)(cube % m), (int)((cube / m) % m), D == 3 ? (int)(cube / ((int64_t)m * m)) : 0};
  bool any = false;
  for (int b = 0; b < (1 << D); ++b) {
    const int i[3] = {cm[0] + (b & 1), cm[1] + ((b >> 1) & 1), cm[2] + ((b >> 2) & 1)};
    any = any || (flag[smp_node(i, a.n, D)] & 1);
  }
  if (!any) return false;
  for (int b = 0; b < (1 << D); ++b) {
    const int i[3] = {cm[0] + (b & 1), cm[1] + ((b >> 1) & 1), cm[2] + ((b >> 2) & 1)};
    cphi[b] = phi[smp_node(i, a.n, D)];
    for (int q = 0; q < 3; ++q) cpos[b][q] = mul_nc((double)i[q] + 0.5, a.dx);
  }
  return true;
}

// Samples of every cube (0 for cubes without an element).
template <int D>
__global__ void k_smp_count(SmpArgs a, const uint8_t* flag, const double* phi, int* cnt_out) {
  const int64_t cube = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = a.n - 1;
  const int64_t ncube = (int64_t)m * m * (D == 3 ? m : 1);
  if (cube >= ncube) return;
  double cphi[8], cpos[8][3];
  int total = 0;
  if (smp_cube<D>(cube, a, flag, phi, cphi, cpos)) {
    for (int t = 0; t < (D == 3 ? 6 : 2); ++t) {
      SmpElem e[2];
      const int ne = smp_simplex<D>(cube, t, cphi, cpos, e);
      for (int k = 0; k < ne; ++k) {
        double nh[3], meas;
        total += (int)smp_measure<D>(e[k], a, nh, &meas);
      }
    }
  }
  cnt_out[cube] = total;
}

// Writes the samples of every cube at its offset, s and dA as [dim][total] (total =
// off[ncube]), when total <= cap.
template <int D, typename R>
__global__ void k_smp_emit(SmpArgs a, const uint8_t* flag, const double* phi, const int* cnt, const int* off,
                           int64_t cap, R* s, R* dA, int* label) {
  const int64_t cube = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = a.n - 1;
  const int64_t ncube = (int64_t)m * m * (D == 3 ? m : 1);
  if (cube >= ncube || cnt[cube] == 0) return;
  const int64_t total = off[ncube];
  if (total > cap) return;
  double cphi[8], cpos[8][3];
  if (!smp_cube<D>(cube, a, flag, phi, cphi, cpos)) return;
  int64_t out = off[cube];
  for (int t = 0; t < (D == 3 ? 6 : 2); ++t) {
    SmpElem e[2];
    const int ne = smp_simplex<D>(cube, t, cphi, cpos, e);
    for (int k = 0; k < ne; ++k) {
      double nh[3], meas;
      const int64_t c = smp_measure<D>(e[k], a, nh, &meas);
      if (c == 0) continue;
      const double share = meas / (double)c;
      for (int64_t j = 0; j < c; ++j, ++out) {
        double q[3] = {0, 0, 0};
        if (D == 3) {
          const double r1 = smp_draw(a.key, (uint64_t)e[k].id, 1 + 2 * j);
          const double r2 = smp_draw(a.key, (uint64_t)e[k].id, 2 + 2 * j);
          const double sq = sqrt(r1);
          const double w0 = sub_nc(1.0, sq), w1 = mul_nc(sq, sub_nc(1.0, r2)), w2 = mul_nc(sq, r2);
          for (int g = 0; g < 3; ++g)
            q[g] = add_nc(add_nc(mul_nc(w0, e[k].v[0][g]), mul_nc(w1, e[k].v[1][g])),
                             mul_nc(w2, e[k].v[2][g]));
        } else {
          const double r1 = smp_draw(a.key, (uint64_t)e[k].id, 1 + j);
          for (int g = 0; g < 2; ++g)
            q[g] = add_nc(e[k].v[0][g], mul_nc(r1, sub_nc(e[k].v[1][g], e[k].v[0][g])));
        }
        bool in = a.has_label;
        for (int g = 0; g < D; ++g) {
          s[(int64_t)g * total + out] = (R)q[g];
          dA[(int64_t)g * total + out] = (R)mul_nc(nh[g], share);
          if (in) in = q[g] >= a.lo[g] && q[g] < a.hi[g];
        }
        if (label) label[out] = in ? 1 : 0;
      }
    }
  }
}

}  // namespace mpm
