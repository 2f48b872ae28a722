// Host input stage (Section 4.1.1): surface samples of the union-of-spheres level set.
//
// phi(x) = min_p |x - x_p| - r is evaluated exactly at the corners of every lattice cube
// that has a corner inside (phi < 0); the zero isocontour is extracted by marching
// tetrahedra (six tets around each cube's main diagonal, 3D) or marching triangles (two
// per square, 2D); each element of measure A receives max(1, floor(density A + u))
// uniform samples (Osada's square-root barycentric map in 3D), each with dA equal to the
// outward unit normal times A / count.  Random numbers are SplitMix64 outputs used as a
// counter-based generator: element id e, draw j -> mix(mix(key + (e+1) G) + (j+1) G),
// key = seed * 2^32 + step, G = 0x9E3779B97F4A7C15; the top 53 bits scaled by 2^-53.
// Element ids: cube c = i0 + (n-1)(i1 + (n-1) i2), id = (c * T + t) * 2 + j, T = 6 tets or
// 2 triangles per cube, j the element within the tet / triangle.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/mpm.h"

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline double draw(uint64_t key, uint64_t elem, uint64_t j) {
  uint64_t s = mix64(key + (elem + 1) * kGolden);
  uint64_t z = mix64(s + (j + 1) * kGolden);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

struct Grid {
  int dim, n;
  double dx;
  std::vector<int> start, order;   // particles binned by cell (natural order)
  const double* x;
  int64_t np;
  int64_t cell(const int* c) const { return c[0] + (int64_t)n * (c[1] + (dim == 3 ? (int64_t)n * c[2] : 0)); }
};

void bin(Grid& g) {
  int64_t nc = 1;
  for (int a = 0; a < g.dim; ++a) nc *= g.n;
  std::vector<int64_t> key(g.np);
  g.start.assign(nc + 1, 0);
  for (int64_t p = 0; p < g.np; ++p) {
    int c[3] = {0, 0, 0};
    for (int a = 0; a < g.dim; ++a) {
      double v = std::floor(g.x[a * g.np + p] / g.dx);
      c[a] = (int)std::min<double>(std::max<double>(v, 0.0), g.n - 1);
    }
    key[p] = g.cell(c);
    g.start[key[p] + 1]++;
  }
  for (int64_t c = 0; c < nc; ++c) g.start[c + 1] += g.start[c];
  g.order.resize(g.np);
  std::vector<int> cur(g.start.begin(), g.start.end() - 1);
  for (int64_t p = 0; p < g.np; ++p) g.order[cur[key[p]]++] = (int)p;
}

// Exact nearest-particle distance of node i over the particles in the cells within 3
// cells of the node's cell (the level set is only needed near the particles).  Searched
// in shells of growing Chebyshev radius R: every particle outside the shells searched so
// far is at least (R + 1/2) dx away (the node sits at its cell's centre), so the search
// stops once the best distance is within that bound; the minimum is the same as the
// full 7^d search.
double node_dist(const Grid& g, const int* i) {
  double pos[3] = {0, 0, 0};
  for (int a = 0; a < g.dim; ++a) pos[a] = (i[a] + 0.5) * g.dx;
  double best = 1e300;
  auto visit_cell = [&](const int* c) {
    int64_t ci = g.cell(c);
    for (int k = g.start[ci]; k < g.start[ci + 1]; ++k) {
      int p = g.order[k];
      double d2 = 0;
      for (int a = 0; a < g.dim; ++a) {
        double t = pos[a] - g.x[a * g.np + p];
        d2 += t * t;
      }
      best = std::min(best, d2);
    }
  };
  for (int R = 0; R <= 3; ++R) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < g.dim; ++a) { lo[a] = std::max(i[a] - R, 0); hi[a] = std::min(i[a] + R, g.n - 1); }
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          int c[3] = {x, y, z};
          int ring = 0;
          for (int a = 0; a < g.dim; ++a) ring = std::max(ring, std::abs(c[a] - i[a]));
          if (ring == R) visit_cell(c);
        }
    const double bound = (R + 0.5) * g.dx;
    if (best <= bound * bound) break;
  }
  return std::sqrt(best);
}

struct Elem {
  int64_t id;
  double v[3][3];
  double ori[3];
};

const int kTets[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};
const int kTris[2][3] = {{0, 1, 3}, {0, 3, 2}};

void edge_point(const double* xu, const double* xv, double pu, double pv, int dim, double* out) {
  double t = pu / (pu - pv);
  for (int a = 0; a < dim; ++a) out[a] = xu[a] + t * (xv[a] - xu[a]);
}

}  // namespace

extern "C" int mpm_sample_surface(int32_t dim, int32_t n, const double* x, int64_t n_part, double radius,
                                  double density, uint64_t seed, uint64_t step, const double* label_lo,
                                  const double* label_hi, double* s, double* dA, int32_t* label, int64_t cap,
                                  int64_t* out_n) {
  if ((dim != 2 && dim != 3) || n < 4 || n_part < 0 || (n_part > 0 && !x) || !out_n || cap < 0) return MPM_EINVAL;
  if (cap > 0 && (!s || !dA)) return MPM_EINVAL;
  const double dx = 1.0 / n;
  const double r = radius > 0 ? radius : (dim == 3 ? 0.867 : 0.73) * dx;
  const double rho = density > 0 ? density : (dim == 3 ? 8.0 / (dx * dx) : 4.0 / dx);
  *out_n = 0;
  if (n_part == 0) return MPM_OK;
  Grid g{dim, n, dx, {}, {}, x, n_part};
  bin(g);
  const int64_t nn = dim == 3 ? (int64_t)n * n * n : (int64_t)n * n;
  const int m = n - 1;
  const int64_t ncube = dim == 3 ? (int64_t)m * m * m : (int64_t)m * m;
  // inside nodes: some particle closer than r
  std::vector<uint8_t> inside(nn, 0);
  for (int64_t p = 0; p < n_part; ++p) {
    int base[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) base[a] = (int)std::floor(x[a * n_part + p] / dx - 0.5);
    for (int dz = 0; dz <= (dim == 3 ? 1 : 0); ++dz)
      for (int dy = 0; dy <= 1; ++dy)
        for (int dxo = 0; dxo <= 1; ++dxo) {
          int i[3] = {base[0] + dxo, base[1] + dy, base[2] + dz};
          bool ok = true;
          for (int a = 0; a < dim; ++a) ok = ok && i[a] >= 0 && i[a] < n;
          if (!ok) continue;
          double d2 = 0;
          for (int a = 0; a < dim; ++a) {
            double t = (i[a] + 0.5) * dx - x[a * n_part + p];
            d2 += t * t;
          }
          if (std::sqrt(d2) - r < 0) inside[g.cell(i)] = 1;
        }
  }
  // nodes at distance < r from a particle all lie in the 2^d box around it (r < dx);
  // phi's sign is then exact.  Candidate cubes: those with an inside corner.
  std::vector<uint8_t> cand(ncube, 0);
  for (int64_t k = 0; k < nn; ++k) {
    if (!inside[k]) continue;
    int i[3] = {(int)(k % n), (int)((k / n) % n), dim == 3 ? (int)(k / ((int64_t)n * n)) : 0};
    for (int dz = -(dim == 3); dz <= 0; ++dz)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dxo = -1; dxo <= 0; ++dxo) {
          int c[3] = {i[0] + dxo, i[1] + dy, i[2] + dz};
          bool ok = true;
          for (int a = 0; a < dim; ++a) ok = ok && c[a] >= 0 && c[a] < m;
          if (!ok) continue;
          cand[c[0] + (int64_t)m * (c[1] + (dim == 3 ? (int64_t)m * c[2] : 0))] = 1;
        }
  }
  std::vector<double> phi(nn, std::nan(""));
  auto phi_at = [&](const int* i) {
    int64_t k = g.cell(i);
    if (std::isnan(phi[k])) phi[k] = node_dist(g, i) - r;
    return phi[k];
  };
  std::vector<Elem> elems;
  const int ncorner = 1 << dim;
  const int T = dim == 3 ? 6 : 2;
  for (int64_t cube = 0; cube < ncube; ++cube) {
    if (!cand[cube]) continue;
    int cm[3] = {(int)(cube % m), (int)((cube / m) % m), dim == 3 ? (int)(cube / ((int64_t)m * m)) : 0};
    double cphi[8], cpos[8][3];
    int nneg = 0;
    for (int b = 0; b < ncorner; ++b) {
      int i[3] = {cm[0] + (b & 1), cm[1] + ((b >> 1) & 1), cm[2] + ((b >> 2) & 1)};
      cphi[b] = phi_at(i);
      for (int a = 0; a < 3; ++a) cpos[b][a] = (i[a] + 0.5) * dx;
      nneg += cphi[b] < 0;
    }
    if (nneg == 0 || nneg == ncorner) continue;
    for (int t = 0; t < T; ++t) {
      const int nv = dim + 1;
      int vid[4];
      for (int k = 0; k < nv; ++k) vid[k] = dim == 3 ? kTets[t][k] : kTris[t][k];
      double sp[4];
      bool neg[4];
      int cnt = 0;
      double mo[3] = {0, 0, 0}, mi[3] = {0, 0, 0};
      int no = 0, ni = 0;
      for (int k = 0; k < nv; ++k) {
        sp[k] = cphi[vid[k]];
        neg[k] = sp[k] < 0;
        cnt += neg[k];
        for (int a = 0; a < dim; ++a) (neg[k] ? mi : mo)[a] += cpos[vid[k]][a];
        (neg[k] ? ni : no)++;
      }
      if (cnt == 0 || cnt == nv) continue;
      double ori[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) ori[a] = mo[a] / no - mi[a] / ni;
      const int64_t base_id = (cube * T + t) * 2;
      auto P = [&](int u, int v, double* out) { edge_point(cpos[vid[u]], cpos[vid[v]], sp[u], sp[v], dim, out); };
      if (dim == 3) {
        if (cnt == 1 || cnt == 3) {
          bool lone_in = cnt == 1;
          int a = 0;
          while ((neg[a] != lone_in)) ++a;
          Elem e{base_id, {}, {ori[0], ori[1], ori[2]}};
          int q = 0;
          for (int k = 0; k < 4; ++k) {
            if (k == a) continue;
            if (lone_in) P(a, k, e.v[q]); else P(k, a, e.v[q]);
            ++q;
          }
          elems.push_back(e);
        } else {
          int ins[2], outs[2], qi = 0, qo = 0;
          for (int k = 0; k < 4; ++k) { if (neg[k]) ins[qi++] = k; else outs[qo++] = k; }
          double pac[3], pad[3], pbd[3], pbc[3];
          P(ins[0], outs[0], pac); P(ins[0], outs[1], pad); P(ins[1], outs[1], pbd); P(ins[1], outs[0], pbc);
          Elem e0{base_id, {}, {ori[0], ori[1], ori[2]}}, e1{base_id + 1, {}, {ori[0], ori[1], ori[2]}};
          std::memcpy(e0.v[0], pac, sizeof pac); std::memcpy(e0.v[1], pad, sizeof pad); std::memcpy(e0.v[2], pbd, sizeof pbd);
          std::memcpy(e1.v[0], pac, sizeof pac); std::memcpy(e1.v[1], pbd, sizeof pbd); std::memcpy(e1.v[2], pbc, sizeof pbc);
          elems.push_back(e0);
          elems.push_back(e1);
        }
      } else {
        bool lone_in = cnt == 1;
        int a = 0;
        while ((neg[a] != lone_in)) ++a;
        Elem e{base_id, {}, {ori[0], ori[1], 0}};
        int q = 0;
        for (int k = 0; k < 3; ++k) {
          if (k == a) continue;
          if (lone_in) P(a, k, e.v[q]); else P(k, a, e.v[q]);
          ++q;
        }
        elems.push_back(e);
      }
    }
  }
  const uint64_t key = (seed << 32) + step;
  int64_t out = 0;
  for (const Elem& e : elems) {
    double nv[3] = {0, 0, 0}, meas;
    if (dim == 3) {
      double u[3], w[3];
      for (int a = 0; a < 3; ++a) { u[a] = e.v[1][a] - e.v[0][a]; w[a] = e.v[2][a] - e.v[0][a]; }
      nv[0] = u[1] * w[2] - u[2] * w[1];
      nv[1] = u[2] * w[0] - u[0] * w[2];
      nv[2] = u[0] * w[1] - u[1] * w[0];
      meas = 0.5 * std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    } else {
      double ex = e.v[1][0] - e.v[0][0], ey = e.v[1][1] - e.v[0][1];
      nv[0] = -ey;
      nv[1] = ex;
      meas = std::sqrt(ex * ex + ey * ey);
    }
    if (!(meas > 0)) continue;
    double nl = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    double nh[3] = {nv[0] / nl, nv[1] / nl, nv[2] / nl};
    double dot = 0;
    for (int a = 0; a < dim; ++a) dot += nh[a] * e.ori[a];
    if (dot < 0)
      for (int a = 0; a < 3; ++a) nh[a] = -nh[a];
    double u0 = draw(key, (uint64_t)e.id, 0);
    int64_t cnt = std::max<int64_t>(1, (int64_t)std::floor(rho * meas + u0));
    for (int64_t j = 0; j < cnt; ++j, ++out) {
      if (out >= cap) continue;
      double q[3];
      if (dim == 3) {
        double r1 = draw(key, (uint64_t)e.id, 1 + 2 * j), r2 = draw(key, (uint64_t)e.id, 2 + 2 * j);
        double sq = std::sqrt(r1);
        for (int a = 0; a < 3; ++a) q[a] = (1 - sq) * e.v[0][a] + (sq * (1 - r2)) * e.v[1][a] + (sq * r2) * e.v[2][a];
      } else {
        double r1 = draw(key, (uint64_t)e.id, 1 + j);
        for (int a = 0; a < 2; ++a) q[a] = e.v[0][a] + r1 * (e.v[1][a] - e.v[0][a]);
      }
      bool in = label_lo && label_hi;
      for (int a = 0; a < dim; ++a) {
        s[a * cap + out] = q[a];
        dA[a * cap + out] = nh[a] * (meas / cnt);
        if (in) in = q[a] >= label_lo[a] && q[a] < label_hi[a];
      }
      if (label) label[out] = in ? 1 : 0;
    }
  }
  *out_n = out;
  return MPM_OK;
}
