// Cell-tile kernels: the scatter halves of P2G, the energy gradient, the Hessian-vector
// product and the heat operator.
//
// One workgroup owns one tile of cells (4x4x4 in 3D, 8x8 in 2D).  Its points (interior
// particles, surface samples, balance points: contiguous ranges after the cell sort) are
// staged through LDS in chunks.  The point phase gathers what it needs from the tile's
// node region (6^3 / 10^2 nodes, staged in LDS) and stores a per-point payload; the
// scatter phase maps lanes to (cell, k0, k1): each lane accumulates, in registers and in
// the fixed order of the cell's points, the contributions to the 3 nodes
// (c0-1+k0, c1-1+k1, c2-1+k2), k2 = 0..2 (3D) or to the 3 nodes along k1 (2D).  The 3D
// stress and heat kernels gather from, and scatter into, per-plane polynomial coefficients
// of the region instead (mono_build, mono_grad, lane_scatter_mono): their lanes stand for
// (cell, component, z plane) and map their sums to the plane patch's nodes at the end.  The
// per-cell partials are then reduced in LDS, in fixed order, onto the node region, which
// is written to a per-tile partial buffer.  A merge kernel sums, for every node, the
// partials of the <= 2^d tiles whose region holds it (fixed order) and applies the
// node-level terms.  No float atomics anywhere: results are bitwise reproducible.
#pragma once
#include <type_traits>
#include "kernels.h"

namespace mpm {

// Tile kernels run 9-wave (3D) workgroups.  The dispatcher places three waves of every
// such workgroup on one SIMD, so k resident workgroups need 3k wave slots on that SIMD:
// two per CU fit at most 85 VGPRs (80 allocated), three need at most 56.  The kernels
// ask for W waves per SIMD; the compiler honours that only while its own LDS estimate
// allows W, so the static LDS of a block stays under a third of the CU's 160 KB (the
// stress kernel, larger, takes dynamic LDS, which the estimate does not see).  P2G fits 73
// (MIXED) by itself.  FP64 kernels need about twice the registers: at one workgroup per
// CU they ask for 3 or 4 waves per SIMD (up to 168 or 128 VGPRs); held to 80, the FP64
// stress and heat kernels spilled over 300 bytes per lane.
#define MPM_TILE_KERNEL(NT, W) __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(W)))
template <typename R> struct TileOcc;
template <> struct TileOcc<float> { static constexpr int STRESS = 6, HEAT = 6, P2G = 6; };
template <> struct TileOcc<double> { static constexpr int STRESS = 3, HEAT = 3, P2G = 4; };

template <int D> struct TileGeo;
template <> struct TileGeo<3> {
  static constexpr int E = 4;          // cells per tile edge
  static constexpr int RE = 6;         // node-region edge (E + 2)
  static constexpr int RN = 216;       // region nodes
  static constexpr int LPC = 9;        // scatter lanes per cell (k0, k1)
  static constexpr int NT = 576;       // threads per workgroup (64 cells x 9)
};
template <> struct TileGeo<2> {
  static constexpr int E = 8;
  static constexpr int RE = 10;
  static constexpr int RN = 100;
  static constexpr int LPC = 3;        // (k0), k1 looped
  static constexpr int NT = 192;
};

// Device view of the tile lists.
struct TileLists {
  const int* ctile_list;   // active cell tiles (compact)
  const int* ctile_slot;   // cell tile -> slot in ctile_list, -1 when inactive
  const int* ctile_rng;    // per slot: [interior begin, end, surface begin, end, balance begin, end]
  const int* nbr;          // per active node tile ti: slots of the cell tiles at offsets -1..1 (kNbr)
  int nctile;
  int xrun;                // slots per XCD run of the tile kernels (xcd_slot)
};

// Slot of the tile that workgroup b takes.  Workgroups are dealt to the 8 XCDs in turn,
// and each XCD has an L2 of its own; neighbouring cell tiles (consecutive slots) read
// overlapping node regions, so each XCD takes runs of `run` consecutive slots, the runs
// dealt to the XCDs in turn.  The halo lines a tile shares with the previous one are then
// in its own XCD's L2.  A launch covers whole rounds of 8 runs (xcd_grid); workgroups past
// the last slot return.
MPM_DEV int xcd_slot(int b, int run) {
  const int x = b & 7, i = b >> 3;
  return (i / run) * (8 * run) + x * run + (i % run);
}
inline int xcd_grid(int nslot, int run) { return (nslot + 8 * run - 1) / (8 * run) * 8 * run; }
inline int xcd_run(int nslot) { return nslot >= 8192 ? 32 : (nslot >= 1024 ? 8 : 1); }

constexpr int kNbr = 27;   // neighbour slots per node tile (3^D used)

template <int D>
struct MergeSrc {
  int slot[1 << D];   // partial slot of candidate j, -1 if absent
  int rn[1 << D];     // node's index in that tile's region
};

// The cell tiles whose 6^3 (10^2) node regions contain a node: its own tile and, on a
// tile face, the neighbour across it.  Candidate j (0 <= j < 2^D, axis a taking the
// bit k_a of j, higher axes outer) is the tile base_a + k_a per axis; the candidates are
// visited in increasing tile coordinates, which fixes the summation order.  Every
// index is a compile-time constant after unrolling, so the arrays stay in registers and
// all slot lookups and partial loads can be in flight together.
template <int D>
MPM_DEV void merge_sources(int node_tile, int local, int nt, const int* ctile_slot, MergeSrc<D>& ms) {
  constexpr int E = TileGeo<D>::E, RE = TileGeo<D>::RE;
  int i[3] = {0, 0, 0};
  tiled_coords<D>(node_tile, local, nt, i);
  int base[3] = {0, 0, 0}, two[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int T = i[a] / E, l = i[a] % E;
    base[a] = l == 0 ? T - 1 : T;
    two[a] = (l == 0 || l == E - 1) ? 1 : 0;
  }
#pragma unroll
  for (int j = 0; j < (1 << D); ++j) {
    int C[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = (j >> a) & 1;
      C[a] = base[a] + k;
      ok = ok && (k == 0 || two[a]) && C[a] >= 0 && C[a] < nt;
    }
    const int ct = C[0] + nt * (C[1] + (D == 3 ? nt * C[2] : 0));
    const int s = ok ? ctile_slot[ct] : -1;
    int r[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = i[a] - (E * C[a] - 1);
    ms.slot[j] = s;
    ms.rn[j] = r[0] + RE * (r[1] + (D == 3 ? RE * r[2] : 0));
  }
}

// merge_sources from the table of neighbour slots of the node tile (tl.nbr, written by
// k_merge_p2g): the candidates and their region indices follow from the node's place in
// its tile alone (offset -1 on a low face, +1 on a high face), so the slot loads need not
// wait for the tile's index.  Same candidates, order and values as merge_sources.
template <int D>
MPM_DEV void merge_sources_tab(int ti, int local, const int* nbr, MergeSrc<D>& ms) {
  constexpr int E = TileGeo<D>::E, RE = TileGeo<D>::RE, L = Tiling<D>::LOG;
  const int l[3] = {local & (E - 1), D == 3 ? (local >> L) & (E - 1) : (local >> L), D == 3 ? (local >> (2 * L)) : 0};
#pragma unroll
  for (int j = 0; j < (1 << D); ++j) {
    int off[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = (j >> a) & 1;
      off[a] = (l[a] == 0 ? -1 : 0) + k;
      ok = ok && (k == 0 || l[a] == 0 || l[a] == E - 1);
    }
    const int idx = (off[0] + 1) + 3 * ((off[1] + 1) + (D == 3 ? 3 * (off[2] + 1) : 0));
    ms.slot[j] = ok ? nbr[ti * kNbr + idx] : -1;
    int r[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = l[a] - E * off[a] + 1;
    ms.rn[j] = r[0] + RE * (r[1] + (D == 3 ? RE * r[2] : 0));
  }
}

// Local coordinates of cell lc (tile-local tiled order) and of region node rn.
template <int D>
MPM_DEV void local_cell(int lc, int* c) {
  constexpr int E = TileGeo<D>::E, L = Tiling<D>::LOG;
  c[0] = lc & (E - 1);
  c[1] = (lc >> L) & (E - 1);
  c[2] = D == 3 ? (lc >> (2 * L)) : 0;
}

template <int D>
MPM_DEV void region_coords(int rn, int* r) {
  constexpr int RE = TileGeo<D>::RE;
  r[0] = rn % RE;
  r[1] = (rn / RE) % RE;
  r[2] = D == 3 ? rn / (RE * RE) : 0;
}

template <int D>
MPM_DEV int region_index(const int* r) {
  constexpr int RE = TileGeo<D>::RE;
  return r[0] + RE * (r[1] + (D == 3 ? RE * r[2] : 0));
}

// The first cell of cell tile `tile` (tiled_coords with local 0), in 32-bit arithmetic.
template <int D>
MPM_DEV void tile_origin(int tile, int nt, int* o) {
  constexpr int L = Tiling<D>::LOG;
  const unsigned t = (unsigned)tile, n = (unsigned)nt;
  const unsigned q = t / n;
  o[0] = (int)(t - q * n) << L;
  if (D == 3) {
    const unsigned q2 = q / n;
    o[1] = (int)(q - q2 * n) << L;
    o[2] = (int)q2 << L;
  } else {
    o[1] = (int)q << L;
  }
}

// Global tiled index (tiled_index) of region node r of the cell tile whose first cell is
// org (region origin = org - 1), -1 outside the grid: 32-bit, one bounds test for all axes.
template <int D>
MPM_DEV int region_node_at(const int* org, const int* r, int n, int nt) {
  constexpr int E = Tiling<D>::E, L = Tiling<D>::LOG;
  const int stride[3] = {1, nt, nt * nt};   // node tiles along each axis
  bool ok = true;
  int tile = 0, local = 0;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const int g = org[b] - 1 + r[b];
    ok = ok && (unsigned)g < (unsigned)n;
    tile += (g >> L) * stride[b];
    local += (g & (E - 1)) << (L * b);
  }
  return ok ? tile * kTileNodes + local : -1;
}

// ---------------------------------------------------------------------------------------
// Scatter engine: lanes (cell, k0[, k1]) accumulate NF fields on their 3 nodes.
//   contrib(q, w, g, out[NF]) adds point q's contribution at one node with weight w and
//   weight gradient g (node-relative offsets known to the lane through kk).
// ---------------------------------------------------------------------------------------
template <int D, typename R, int NF>
struct LaneAcc {
  R v[3][NF];
  MPM_DEV void zero() {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int f = 0; f < NF; ++f) v[k][f] = 0;
  }
};

// Writes the lane accumulators to the per-cell LDS partial buffer (fields f0..f0+FC) and
// reduces them onto the node region: out(rn, f, sum over cells c, offsets k with c + k =
// rn), in a fixed order.  Caller synchronizes around.
template <int D, typename R, int NF, int FC, class Out>
MPM_DEV void reduce_cells_to_region_out(const LaneAcc<D, R, NF>& acc, int f0, R* cellpart, int lane_cell, int lane_k0,
                                        int lane_k1, bool lane_on, Out&& out) {
  constexpr int RN = TileGeo<D>::RN, NT = TileGeo<D>::NT, E = TileGeo<D>::E;
  // cellpart layout: [cell 64][k2 3][k1 3][k0 3][FC]  (3D)  /  [cell 64][k1 3][k0 3][FC] (2D)
  if (lane_on) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int f = 0; f < FC; ++f) {
        if (f0 + f >= NF) continue;
        int kk2 = D == 3 ? k : 0, kk1 = D == 3 ? lane_k1 : k;
        int idx = (((lane_cell * 3 + kk2) * 3 + kk1) * 3 + lane_k0) * FC + f;
        cellpart[idx] = acc.v[k][f0 + f];
      }
  }
  __syncthreads();
  // one (node, field) item per thread: the cells c = r - k in [0, E) are visited in (k2,
  // k1, k0) order with predicated reads, all in flight together
  for (int i = threadIdx.x; i < RN * FC; i += NT) {
    const int rn = i / FC, f = i - rn * FC;
    if (f0 + f >= NF) continue;
    int r[3];
    region_coords<D>(rn, r);
    R s = 0;
#pragma unroll
    for (int k2 = 0; k2 < (D == 3 ? 3 : 1); ++k2) {
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) {
#pragma unroll
        for (int k0 = 0; k0 < 3; ++k0) {
          const int c0 = r[0] - k0, c1 = r[1] - k1, c2 = D == 3 ? r[2] - k2 : 0;
          const bool in = c0 >= 0 && c0 < E && c1 >= 0 && c1 < E && c2 >= 0 && c2 < (D == 3 ? E : 1);
          int cc[3] = {in ? c0 : 0, in ? c1 : 0, in ? c2 : 0};
          const int lc = (int)tiled_index<D>(cc, 1) & 63;
          const int base = ((lc * 3 + (D == 3 ? k2 : 0)) * 3 + k1) * 3 + k0;
          s += in ? cellpart[base * FC + f] : R(0);
        }
      }
    }
    out(rn, f, s);
  }
  __syncthreads();
}

// The node terms of a plane patch from the coefficient sensitivities: g_ij = sum_pq
// T_pi T_qj h_pq, with c_p = sum_i T_pi u_i the coefficient map of mono_build
// (T = [[1/2, 1/2, 0], [-1, 1, 0], [1/2, -1, 1/2]]).
template <typename R>
MPM_DEV void mono_unmap(const R (&h)[3][3], R (&g)[3][3]) {
  R m[3][3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    m[0][q] = R(0.5) * (h[0][q] + h[2][q]) - h[1][q];
    m[1][q] = R(0.5) * h[0][q] + h[1][q] - h[2][q];
    m[2][q] = R(0.5) * h[2][q];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g[i][0] = R(0.5) * (m[i][0] + m[i][2]) - m[i][1];
    g[i][1] = R(0.5) * m[i][0] + m[i][1] - m[i][2];
    g[i][2] = R(0.5) * m[i][2];
  }
}

// The same reduction over a dense buffer B[rn][f][k] (k = k0 + 3 k1 + 9 k2, stride KS):
// every (node, offset) slot that no cell of the tile reaches holds zero, so each node's
// sum runs over all 3^D slots in k order without a predicate, and gives the same value as
// the predicated form (the skipped terms are added as zeros there).  The buffer shares its
// storage with the point payloads, so it is cleared first.  out(rn, f, v) receives the
// sums.
template <int D>
struct DenseRed {
  static constexpr int KN = D == 3 ? 27 : 9;
  static constexpr int KS = (KN + 3) & ~3;   // whole 16-byte rows
};

template <int D, typename R, int NF, class Out, bool MONO = false, class Acc>
MPM_DEV void reduce_region_dense(const Acc& acc, R* B, int lane_cell, int lane_k0, int lane_k1, bool lane_on,
                                 Out&& out) {
  constexpr int RN = TileGeo<D>::RN, RE = TileGeo<D>::RE, NT = TileGeo<D>::NT, KN = DenseRed<D>::KN,
                KS = DenseRed<D>::KS;
  constexpr int NB = RN * NF * KS;
  static_assert((NB * sizeof(R)) % 16 == 0, "whole 16-byte rows");
  uint4* B16 = reinterpret_cast<uint4*>(B);   // all-zero bits are 0.0 in both precisions
  for (int i = threadIdx.x; i < (int)(NB * sizeof(R) / 16); i += NT) B16[i] = make_uint4(0, 0, 0, 0);
  __syncthreads();
  if (lane_on) {
    int c[3];
    local_cell<D>(lane_cell, c);
    if constexpr (MONO) {
      // lane (component lane_k0, plane lane_k1): its coefficient sensitivities to the
      // nodes of its plane patch (lane_scatter_mono)
      static_assert(D == 3 && (NF == 3 || NF == 1), "plane patches of the 3D scatters");
      R g[3][3];
      mono_unmap<R>(acc.v, g);
      const int a = lane_k0, kz = lane_k1;
      // slot (node c + (i, j, kz), field a, offset i + 3 j + 9 kz): one base index and
      // compile-time steps along i and j
      const int r0[3] = {c[0], c[1], c[2] + kz};
      const int base = (region_index<D>(r0) * NF + a) * KS + 9 * kz;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) B[base + i * (NF * KS + 1) + j * (RE * NF * KS + 3)] = g[i][j];
    } else {
      // slot (node c + (k0, k1, k) in 3D or c + (k0, k) in 2D, field f, offset k0 + 3 k1 +
      // 9 k2): one base index and compile-time steps along k and f
      const int r0[3] = {c[0] + lane_k0, c[1] + (D == 3 ? lane_k1 : 0), D == 3 ? c[2] : 0};
      const int base = region_index<D>(r0) * NF * KS + lane_k0 + (D == 3 ? 3 * lane_k1 : 0);
      constexpr int step = D == 3 ? RE * RE * NF * KS + 9 : RE * NF * KS + 3;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int f = 0; f < NF; ++f) B[base + k * step + f * KS] = acc.v[k][f];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < RN * NF; i += NT) {
    const R* b = B + i * KS;
    R v[KN];
#pragma unroll
    for (int k = 0; k < KN; ++k) v[k] = b[k];
    R sum = 0;
#pragma unroll
    for (int k = 0; k < KN; ++k) sum += v[k];
    out(i / NF, i - (i / NF) * NF, sum);
  }
  __syncthreads();
}

// Lane mapping of the scatter phase.
template <int D>
MPM_DEV void lane_map(int t, int& cell, int& k0, int& k1) {
  if constexpr (D == 3) {
    cell = t / 9;
    k0 = t % 3;
    k1 = (t / 3) % 3;
  } else {
    cell = t / 3;
    k0 = t % 3;
    k1 = 0;
  }
}

// Weight / gradient of the lane's node number k (k2 in 3D, k1 in 2D) from cell-relative f.
template <int D, typename R>
MPM_DEV R lane_weight(const R* f, int k0, int k1, int k, R fn, R* g) {
  int kk[3] = {k0, D == 3 ? k1 : k, D == 3 ? k : 0};
  return weight_from_cell<D, R>(kk, f, fn, g);
}

// Surface derivative Q = d|cof(F) N|/dF (HESS = false) or its linearization along
// dG = dt G (HESS = true, PSD part plus the indefinite part when exact); returns |cof(F) N|.
template <int D, typename R>
MPM_DEV R surface_q(const R (&F)[D][D], const R* Nv, bool hess, const R (&G)[D][D], R dt, int exact, R (&Q)[D][D]) {
  if constexpr (D == 3) {
    R av[3] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      int p = (m + 1) % 3, q = (m + 2) % 3;
      R cx = F[1][p] * F[2][q] - F[2][p] * F[1][q];
      R cy = F[2][p] * F[0][q] - F[0][p] * F[2][q];
      R cz = F[0][p] * F[1][q] - F[1][p] * F[0][q];
      av[0] += cx * Nv[m]; av[1] += cy * Nv[m]; av[2] += cz * Nv[m];
    }
    R an = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
    R ah[3] = {av[0] / an, av[1] / an, av[2] / an};
    R uu[3] = {ah[0], ah[1], ah[2]};
    R dG[3][3];
    if (hess) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) dG[a][b] = dt * G[a][b];
      R da[3] = {0, 0, 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        R dg1[3] = {dG[0][k1], dG[1][k1], dG[2][k1]}, dg2[3] = {dG[0][k2], dG[1][k2], dG[2][k2]};
        R g1[3] = {F[0][k1], F[1][k1], F[2][k1]}, g2[3] = {F[0][k2], F[1][k2], F[2][k2]};
        R c1[3], c2[3];
        cross3<R>(dg1, g2, c1);
        cross3<R>(g1, dg2, c2);
#pragma unroll
        for (int a = 0; a < 3; ++a) da[a] += Nv[k] * (c1[a] + c2[a]);
      }
      R ad = ah[0] * da[0] + ah[1] * da[1] + ah[2] * da[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) uu[a] = (da[a] - ah[a] * ad) / an;
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      int m1 = (m + 1) % 3, m2 = (m + 2) % 3;
      R gp[3] = {F[0][m1], F[1][m1], F[2][m1]}, gq[3] = {F[0][m2], F[1][m2], F[2][m2]};
      R c1[3], c2[3];
      cross3<R>(gp, uu, c1);
      cross3<R>(uu, gq, c2);
#pragma unroll
      for (int a = 0; a < 3; ++a) Q[a][m] = Nv[m2] * c1[a] + Nv[m1] * c2[a];
      if (hess && exact) {
        R dp[3] = {dG[0][m1], dG[1][m1], dG[2][m1]}, dq[3] = {dG[0][m2], dG[1][m2], dG[2][m2]};
        cross3<R>(dp, ah, c1);
        cross3<R>(ah, dq, c2);
#pragma unroll
        for (int a = 0; a < 3; ++a) Q[a][m] += Nv[m2] * c1[a] + Nv[m1] * c2[a];
      }
    }
    return an;
  } else {
    R tau[2] = {Nv[1], -Nv[0]};
    R cv[2] = {F[0][0] * tau[0] + F[0][1] * tau[1], F[1][0] * tau[0] + F[1][1] * tau[1]};
    R cn = sqrt(cv[0] * cv[0] + cv[1] * cv[1]);
    R ch[2] = {cv[0] / cn, cv[1] / cn};
    R uu[2] = {ch[0], ch[1]};
    if (hess) {
      R dc[2] = {dt * (G[0][0] * tau[0] + G[0][1] * tau[1]), dt * (G[1][0] * tau[0] + G[1][1] * tau[1])};
      R cd = ch[0] * dc[0] + ch[1] * dc[1];
      uu[0] = (dc[0] - ch[0] * cd) / cn;
      uu[1] = (dc[1] - ch[1] * cd) / cn;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) Q[a][b] = uu[a] * tau[b];
    // |cof(F) N| = |F tau| in 2D
    return cn;
  }
}

// ======================================================================================
// Stress scatter: energy gradient (ENERGY), Hessian-vector product (HESS) or the force
// of a given velocity field (FORCE, no energy).  Output: per-tile partial of
// sum_q S_q grad N_i over the region (D components per node).
// ======================================================================================
enum TileMode { TM_ENERGY = 0, TM_HESS = 1, TM_FORCE = 2 };

// Per-point 1D weight table: w[a][k], dw[a][k] (dw per unit length) for the nodes
// c_a - 1 + k of the point's stencil.
template <int D, typename R>
MPM_DEV void weight_table(const R* f, R fn, R (&w)[D][3], R (&dw)[D][3]) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    R x = f[a];
    w[a][0] = R(0.5) * (R(1) - x) * (R(1) - x);
    w[a][1] = R(0.75) - (x - R(0.5)) * (x - R(0.5));
    w[a][2] = R(0.5) * x * x;
    dw[a][0] = (x - R(1)) * fn;
    dw[a][1] = (R(1) - R(2) * x) * fn;
    dw[a][2] = x * fn;
  }
}

// Gradient sum_k u_a[k] grad N_k of NC components staged on the region (u[rn*NC + a]) by
// sum factorization over the axes (the tensor-product structure of N).
template <int D, typename R, int NC>
MPM_DEV void region_grad(const R* u, const int* lc, const R (&w)[D][3], const R (&dw)[D][3], R (&G)[NC][D],
                         R* val) {
  constexpr int RE = TileGeo<D>::RE;
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    val[a] = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) G[a][b] = 0;
  }
  if constexpr (D == 3) {
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) {
      R A[NC], B[NC], Cc[NC], V[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) { A[a] = 0; B[a] = 0; Cc[a] = 0; V[a] = 0; }
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) {
        int base = lc[0] + RE * ((lc[1] + k1) + RE * (lc[2] + k2));
#pragma unroll
        for (int a = 0; a < NC; ++a) {
          R u0 = u[(base + 0) * NC + a], u1 = u[(base + 1) * NC + a], u2 = u[(base + 2) * NC + a];
          R s = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
          R sd = u0 * dw[0][0] + u1 * dw[0][1] + u2 * dw[0][2];
          A[a] += sd * w[1][k1];
          B[a] += s * dw[1][k1];
          Cc[a] += s * w[1][k1];
        }
      }
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        G[a][0] += A[a] * w[2][k2];
        G[a][1] += B[a] * w[2][k2];
        G[a][2] += Cc[a] * dw[2][k2];
        val[a] += Cc[a] * w[2][k2];
      }
    }
  } else {
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      int base = lc[0] + RE * (lc[1] + k1);
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        R u0 = u[(base + 0) * NC + a], u1 = u[(base + 1) * NC + a], u2 = u[(base + 2) * NC + a];
        R s = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
        R sd = u0 * dw[0][0] + u1 * dw[0][1] + u2 * dw[0][2];
        G[a][0] += sd * w[1][k1];
        G[a][1] += s * dw[1][k1];
        val[a] += s * w[1][k1];
      }
    }
  }
}

// The trace of region_grad's G for NC = D (the divergence of u), from the diagonal entries
// alone, each formed with region_grad's operations in its order, so the value is the same.
template <int D, typename R>
MPM_DEV R region_div(const R* u, const int* lc, const R (&w)[D][3], const R (&dw)[D][3]) {
  constexpr int RE = TileGeo<D>::RE;
  R Gd[D];
#pragma unroll
  for (int a = 0; a < D; ++a) Gd[a] = 0;
  if constexpr (D == 3) {
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) {
      R A0 = 0, B1 = 0, C2 = 0;
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) {
        int base = lc[0] + RE * ((lc[1] + k1) + RE * (lc[2] + k2));
        {
          R u0 = u[(base + 0) * 3 + 0], u1 = u[(base + 1) * 3 + 0], u2 = u[(base + 2) * 3 + 0];
          R sd = u0 * dw[0][0] + u1 * dw[0][1] + u2 * dw[0][2];
          A0 += sd * w[1][k1];
        }
        {
          R u0 = u[(base + 0) * 3 + 1], u1 = u[(base + 1) * 3 + 1], u2 = u[(base + 2) * 3 + 1];
          R sv = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
          B1 += sv * dw[1][k1];
        }
        {
          R u0 = u[(base + 0) * 3 + 2], u1 = u[(base + 1) * 3 + 2], u2 = u[(base + 2) * 3 + 2];
          R sv = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
          C2 += sv * w[1][k1];
        }
      }
      Gd[0] += A0 * w[2][k2];
      Gd[1] += B1 * w[2][k2];
      Gd[2] += C2 * dw[2][k2];
    }
  } else {
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      int base = lc[0] + RE * (lc[1] + k1);
      {
        R u0 = u[(base + 0) * 2 + 0], u1 = u[(base + 1) * 2 + 0], u2 = u[(base + 2) * 2 + 0];
        R sd = u0 * dw[0][0] + u1 * dw[0][1] + u2 * dw[0][2];
        Gd[0] += sd * w[1][k1];
      }
      {
        R u0 = u[(base + 0) * 2 + 1], u1 = u[(base + 1) * 2 + 1], u2 = u[(base + 2) * 2 + 1];
        R sv = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
        Gd[1] += sv * dw[1][k1];
      }
    }
  }
  R tr = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) tr += Gd[a];
  return tr;
}

// 3D stencil sums from polynomial coefficients.  On a cell, the quadratic B-spline weights
// of the nodes c - 1 + k (k = 0..2) at the cell-relative coordinate x sum a nodal line to a
// quadratic in x: sum_k u_k w_k(x) = c0 + c1 x + c2 x^2 with c0 = (u0 + u1)/2, c1 = u1 - u0,
// c2 = (u0 + u2)/2 - u1 (the three weights of weight_table expanded).  Applied along the
// first two axes to the 3x3 node patch of each stencil start (sx, sy) of the tile, in each
// node plane z of the region, this gives 9 coefficients c_pq of x^p y^q per component.  A
// point then forms the value and the x and y derivatives of each of its three planes by
// Horner's rule, and sums the planes with the z weights, where the direct sum runs over
// the 27 nodes with the weight products.  NC components per node.
template <int NC>
struct MonoGeo {
  static constexpr int E = TileGeo<3>::E, RE = TileGeo<3>::RE;
  static constexpr int NS = E * E * RE;        // stencil starts (sx, sy) times node planes z
  static constexpr int CS = (9 * NC + 3) & ~3;  // per start: NC x 9, padded to 16-byte rows
  static constexpr int N = NS * CS;
};

// Coefficients of every start, from the staged region u[rn * NC + a]: one thread per
// (start, component), NC * NS of the workgroup's threads.
template <typename R, int NC>
MPM_DEV void mono_build(const R* u, R* cf) {
  constexpr int E = MonoGeo<NC>::E, RE = MonoGeo<NC>::RE, CS = MonoGeo<NC>::CS;
  const int j = threadIdx.x;
  if (j >= NC * MonoGeo<NC>::NS) return;
  const int s = j / NC, a = j - NC * s;
  const int sx = s % E, sy = (s / E) % E, z = s / (E * E);
  R X[3][3];   // X[p][r]: the x^p coefficient of patch row r
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const R* row = u + (sx + RE * ((sy + r) + RE * z)) * NC + a;
    const R u0 = row[0], u1 = row[NC], u2 = row[2 * NC];
    X[0][r] = R(0.5) * (u0 + u1);
    X[1][r] = u1 - u0;
    X[2][r] = R(0.5) * (u0 + u2) - u1;
  }
  R* o = cf + s * CS + a * 9;
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    o[p * 3 + 0] = R(0.5) * (X[p][0] + X[p][1]);
    o[p * 3 + 1] = X[p][1] - X[p][0];
    o[p * 3 + 2] = R(0.5) * (X[p][0] + X[p][2]) - X[p][1];
  }
}

// One plane's sums for component a of a point at (x, y) in its cell: the value C and the
// derivatives A (along x) and B (along y), per unit of the cell-relative coordinates;
// tx = 2x, ty = 2y.
template <typename R>
MPM_DEV void mono_plane(const R* c, R x, R tx, R y, R ty, R& A, R& B, R& C) {
  R t[3], dd[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    t[q] = fma_r(x, fma_r(x, c[6 + q], c[3 + q]), c[q]);
    dd[q] = fma_r(tx, c[6 + q], c[3 + q]);
  }
  C = fma_r(y, fma_r(y, t[2], t[1]), t[0]);
  B = fma_r(ty, t[2], t[1]);
  A = fma_r(y, fma_r(y, dd[2], dd[1]), dd[0]);
}

// region_grad (3D) from the coefficients: x, y the point's cell-relative coordinates, wz,
// dwz its weight table along z; G the gradient and val the value of each component.
template <typename R, int NC>
MPM_DEV void mono_grad(const R* cf, const int* lc, R x, R y, R fn, const R (&wz)[3], const R (&dwz)[3],
                       R (&G)[NC][3], R (&val)[NC]) {
  constexpr int E = MonoGeo<NC>::E, CS = MonoGeo<NC>::CS;
  const R* base = cf + (lc[0] + E * (lc[1] + E * lc[2])) * CS;
  const R tx = x + x, ty = y + y;
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    val[a] = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) G[a][b] = 0;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R fw = fn * wz[k];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      R A, B, C;
      mono_plane<R>(base + k * E * E * CS + a * 9, x, tx, y, ty, A, B, C);
      G[a][0] = fma_r(A, fw, G[a][0]);
      G[a][1] = fma_r(B, fw, G[a][1]);
      G[a][2] = fma_r(C, dwz[k], G[a][2]);
      val[a] = fma_r(C, wz[k], val[a]);
    }
  }
}

// The trace of mono_grad's G, from the three diagonal entries alone, each formed with
// mono_grad's operations in its order, so the value is the same.
template <typename R>
MPM_DEV R mono_div(const R* cf, const int* lc, R x, R y, R fn, const R (&wz)[3], const R (&dwz)[3]) {
  constexpr int E = MonoGeo<3>::E, CS = MonoGeo<3>::CS;
  const R* base = cf + (lc[0] + E * (lc[1] + E * lc[2])) * CS;
  const R tx = x + x, ty = y + y;
  R Gd[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R fw = fn * wz[k];
    const R* c = base + k * E * E * CS;
    R A, B, C, A1, B1, C1, A2, B2, C2;
    mono_plane<R>(c, x, tx, y, ty, A, B, C);
    mono_plane<R>(c + 9, x, tx, y, ty, A1, B1, C1);
    mono_plane<R>(c + 18, x, tx, y, ty, A2, B2, C2);
    Gd[0] = fma_r(A, fw, Gd[0]);
    Gd[1] = fma_r(B1, fw, Gd[1]);
    Gd[2] = fma_r(C2, dwz[k], Gd[2]);
  }
  R tr = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) tr += Gd[a];
  return tr;
}

// The transpose of the coefficient gather, for the stress scatter (3D).  A lane (cell,
// component a, plane kz) accumulates over its cell's points the sensitivities h_pq of
// that plane's coefficients c_pq of component a to the point terms S_a . grad N:
//   h_pq += gC x^p y^q + gB x^p q y^(q-1) + gA p x^(p-1) y^q,
//   gA = S_a0 fn wz, gB = S_a1 fn wz, gC = S_a2 dwz
// (mono_plane and the plane sums of mono_grad, differentiated by c_pq).
template <typename R>
MPM_DEV void lane_scatter_mono_g(R x, R y, R gA, R gB, R gC, R (&h)[3][3]) {
  const R yy = y * y, xx = x * x, tx = x + x, ty = y + y;
  const R V[3] = {gC, fma_r(gC, y, gB), fma_r(gC, yy, ty * gB)};
  const R U[3] = {gA, gA * y, gA * yy};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    h[0][q] += V[q];
    h[1][q] = fma_r(x, V[q], h[1][q]) + U[q];
    h[2][q] = fma_r(xx, V[q], fma_r(tx, U[q], h[2][q]));
  }
}

// The stress form: fw = fn wz and dwz of the lane's plane, S0..S2 the row a of the stress.
template <typename R>
MPM_DEV void lane_scatter_mono(R x, R y, R fw, R dwz, R S0, R S1, R S2, R (&h)[3][3]) {
  lane_scatter_mono_g<R>(x, y, S0 * fw, S1 * fw, S2 * dwz, h);
}

// Lane (cell, k0[, k1]) view of a point's weights: the weights and gradients of its 3
// nodes k = 0..2 along the last axis.
template <int D, typename R>
MPM_DEV void lane_nodes(const R* W, const R* DW, int k0, int k1, R (&wn)[3], R (&gn)[3][D]) {
  if constexpr (D == 3) {
    R wx = W[0 * 3 + k0], dwx = DW[0 * 3 + k0], wy = W[1 * 3 + k1], dwy = DW[1 * 3 + k1];
    R al = dwx * wy, be = wx * dwy, ga = wx * wy;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R wz = W[2 * 3 + k], dwz = DW[2 * 3 + k];
      wn[k] = ga * wz;
      gn[k][0] = al * wz;
      gn[k][1] = be * wz;
      gn[k][2] = ga * dwz;
    }
  } else {
    R wx = W[k0], dwx = DW[k0];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R wy = W[3 + k], dwy = DW[3 + k];
      wn[k] = wx * wy;
      gn[k][0] = dwx * wy;
      gn[k][1] = wx * dwy;
    }
  }
}

// Derivative (per dx) of the 1D weight of stencil node k at cell-relative x, from X = x fn
// (the point payloads carry X): X - fn, fn - 2 X and X are (x - 1) fn, (1 - 2x) fn and x fn
// of weight_table, bitwise when fn (the grid's n) is a power of two, as scaling by it is
// exact.
template <typename R>
MPM_DEV R bs_dw_fn(int k, R X, R fn) {
  return k == 0 ? X - fn : (k == 1 ? fma_r(X, R(-2), fn) : X);
}

// bs_dw_fn for a node number k that varies across the lanes, without branches: all three
// forms are formed and the lane's is selected.  Held per lane as the two comparisons of k
// (lane masks in scalar registers), so that it takes no vector registers across the
// scatter loop.
template <typename R>
struct LaneDw {
  bool k0, k1;
  MPM_DEV explicit LaneDw(int k) : k0(k == 0), k1(k == 1) {}
  MPM_DEV R operator()(R X, R fn) const { return k0 ? X - fn : (k1 ? fma_r(X, R(-2), fn) : X); }
};

// acc[k][a] += sum_b S[a][b] dN_k/dx_b over the lane's three nodes k (k2 = k in 3D, k1 = k
// in 2D), from the point's scaled cell-relative position F (x fn) and weight table W.  The node
// gradients share the lane's factors (3D: (al wz_k, be wz_k, ga dwz_k) with al = dwx wy,
// be = wx dwy, ga = wx wy), so S g_k = wz_k (al S_.0 + be S_.1) + dwz_k (ga S_.2): 2 FMAs
// per node and component, chained into the accumulator, after a per-point set-up.
template <int D, typename R>
MPM_DEV void lane_scatter_grad(const R* F, const R* W, R fn, int k0, int k1, const LaneDw<R>& d0, const LaneDw<R>& d1,
                               const R (&S)[D][D], R (&acc)[3][D]) {
  if constexpr (D == 3) {
    const R wx = W[k0], dwx = d0(F[0], fn), wy = W[3 + k1], dwy = d1(F[1], fn);
    const R al = dwx * wy, be = wx * dwy, ga = wx * wy;
    R Pa[3], Qa[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Pa[a] = al * S[a][0] + be * S[a][1];
      Qa[a] = ga * S[a][2];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R wz = W[6 + k], dwz = bs_dw_fn<R>(k, F[2], fn);
#pragma unroll
      for (int a = 0; a < 3; ++a) acc[k][a] = fma_r(dwz, Qa[a], fma_r(wz, Pa[a], acc[k][a]));
    }
  } else {
    const R wx = W[k0], dwx = d0(F[0], fn);
    R Pa[2], Qa[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      Pa[a] = dwx * S[a][0];
      Qa[a] = wx * S[a][1];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R wy = W[3 + k], dwy = bs_dw_fn<R>(k, F[1], fn);
#pragma unroll
      for (int a = 0; a < 2; ++a) acc[k][a] = fma_r(dwy, Qa[a], fma_r(wy, Pa[a], acc[k][a]));
    }
  }
}

// lane_scatter_grad for S = s I (the J term alone): the same products and sums with the
// zero entries of S left out.
template <int D, typename R>
MPM_DEV void lane_scatter_iso(const R* F, const R* W, R fn, int k0, int k1, const LaneDw<R>& d0, const LaneDw<R>& d1,
                              R s, R (&acc)[3][D]) {
  if constexpr (D == 3) {
    const R wx = W[k0], dwx = d0(F[0], fn), wy = W[3 + k1], dwy = d1(F[1], fn);
    const R P0 = (dwx * wy) * s, P1 = (wx * dwy) * s, Q2 = (wx * wy) * s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R wz = W[6 + k], dwz = bs_dw_fn<R>(k, F[2], fn);
      acc[k][0] = fma_r(wz, P0, acc[k][0]);
      acc[k][1] = fma_r(wz, P1, acc[k][1]);
      acc[k][2] = fma_r(dwz, Q2, acc[k][2]);
    }
  } else {
    const R wx = W[k0], dwx = d0(F[0], fn);
    const R P0 = dwx * s, Q1 = wx * s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R wy = W[3 + k], dwy = bs_dw_fn<R>(k, F[1], fn);
      acc[k][0] = fma_r(wy, P0, acc[k][0]);
      acc[k][1] = fma_r(dwy, Q1, acc[k][1]);
    }
  }
}

// acc[k][0] += c N_k + q . grad N_k over the lane's three nodes, factored as above.
template <int D, typename R>
MPM_DEV void lane_scatter_heat(const R* F, const R* W, R fn, int k0, int k1, const LaneDw<R>& d0, const LaneDw<R>& d1,
                               R c, const R* q, R (&acc)[3][1]) {
  if constexpr (D == 3) {
    const R wx = W[k0], dwx = d0(F[0], fn), wy = W[3 + k1], dwy = d1(F[1], fn);
    const R al = dwx * wy, be = wx * dwy, ga = wx * wy;
    const R Pv = c * ga + al * q[0] + be * q[1], Qv = ga * q[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k][0] = fma_r(bs_dw_fn<R>(k, F[2], fn), Qv, fma_r(W[6 + k], Pv, acc[k][0]));
  } else {
    const R wx = W[k0], dwx = d0(F[0], fn);
    const R Pv = c * wx + dwx * q[0], Qv = wx * q[1];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k][0] = fma_r(bs_dw_fn<R>(k, F[1], fn), Qv, fma_r(W[3 + k], Pv, acc[k][0]));
  }
}

// LDS of the tile kernels: the point payloads of a chunk and the buffers of the final
// cell-to-region reduction are never live together, so they share storage.  Keeping a
// 9-wave block near 1/3 of the 160 KB lets three blocks (27 of the CU's 32 wave slots)
// reside per CU.
// ---- fixed-corotated solid (Section 3.2.1) ---------------------------------------------
// F_p = (I + dt G) F^n_p with G the velocity gradient at the particle.
template <int D, typename R>
MPM_DEV void solid_F(const Dev<R>& d, int k, const R (&G)[D][D], R dt, R (&F)[D][D]) {
  const int N = d.np;
  R Fn[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) Fn[a][b] = d.pF[(a * D + b) * N + k];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      R acc = Fn[a][b];
#pragma unroll
      for (int c = 0; c < D; ++c) acc += dt * G[a][c] * Fn[c][b];
      F[a][b] = acc;
    }
}

template <int D, typename R>
MPM_DEV R det_of(const R (&F)[D][D]) {
  if constexpr (D == 2) {
    return F[0][0] * F[1][1] - F[0][1] * F[1][0];
  } else {
    return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
           F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  }
}

// cof F = det(F) F^-T.
template <int D, typename R>
MPM_DEV void cofactor_of(const R (&F)[D][D], R (&C)[D][D]) {
  if constexpr (D == 2) {
    C[0][0] = F[1][1]; C[0][1] = -F[1][0];
    C[1][0] = -F[0][1]; C[1][1] = F[0][0];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3, b1 = (b + 1) % 3, b2 = (b + 2) % 3;
        C[a][b] = F[a1][b1] * F[a2][b2] - F[a1][b2] * F[a2][b1];
      }
  }
}

// Orthogonal polar factor R of F (det F > 0): 2D in closed form (the rotation by the
// angle of (F00 + F11, F10 - F01)); 3D by Newton's iteration X <- (X + X^-T) / 2 from X = F,
// which converges quadratically to R, ten steps (singular values within [1/100, 100]).
template <int D, typename R>
MPM_DEV void polar_R(const R (&F)[D][D], R (&Rm)[D][D]) {
  if constexpr (D == 2) {
    const R c = F[0][0] + F[1][1], s = F[1][0] - F[0][1];
    const R h = R(1) / sqrt(c * c + s * s);
    Rm[0][0] = c * h; Rm[0][1] = -s * h;
    Rm[1][0] = s * h; Rm[1][1] = c * h;
  } else {
    R X[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) X[a][b] = F[a][b];
    for (int it = 0; it < 10; ++it) {
      R C[3][3];
      cofactor_of<3, R>(X, C);
      const R inv = R(1) / det_of<3, R>(X);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) X[a][b] = R(0.5) * (X[a][b] + C[a][b] * inv);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) Rm[a][b] = X[a][b];
  }
}

// The solid's stress-scatter matrix dt V0 P F^nT (energy and force modes: P the Piola
// stress at F) or dt V0 dP F^nT (Hessian mode: dP = 2 mu dF + lambda (C : dF) C at the
// cached C = cof F_lin, dF = dt G F^n).  Returns the energy V0 psi(F) in energy mode.
template <int D, typename R, int MODE>
MPM_DEV R solid_stress(const Dev<R>& d, int k, const R (&G)[D][D], R dt, R* fout, R (&Sq)[D][D]) {
  const int N = d.np;
  const R muV = d.pLh[k], lamV = d.pLh[N + k];
  R Fn[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) Fn[a][b] = d.pF[(a * D + b) * N + k];
  R Pm[D][D];
  R e = 0;
  if constexpr (MODE == TM_HESS) {
    const R* cache = d.sF + (size_t)D * D * d.ns;
    R C[D][D], dF[D][D], cdf = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        C[a][b] = cache[(a * D + b) * N + k];
        R acc = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) acc += G[a][c] * Fn[c][b];
        dF[a][b] = dt * acc;
        cdf += C[a][b] * dF[a][b];
      }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) Pm[a][b] = R(2) * muV * dF[a][b] + lamV * cdf * C[a][b];
  } else {
    R F[D][D], Rm[D][D], C[D][D];
    solid_F<D, R>(d, k, G, dt, F);
    polar_R<D, R>(F, Rm);
    cofactor_of<D, R>(F, C);
    const R J = det_of<D, R>(F);
    R fr2 = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const R df = F[a][b] - Rm[a][b];
        fr2 += df * df;
        Pm[a][b] = R(2) * muV * df + lamV * (J - R(1)) * C[a][b];
      }
    e = muV * fr2 + R(0.5) * lamV * (J - R(1)) * (J - R(1));
    if (fout) {
      R* cache = fout + (size_t)D * D * d.ns;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) cache[(a * D + b) * N + k] = C[a][b];
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      R acc = 0;
#pragma unroll
      for (int c = 0; c < D; ++c) acc += Pm[a][c] * Fn[b][c];
      Sq[a][b] = dt * acc;
    }
  return e;
}

// LDS of the stress tile kernel.  The point payloads of a chunk and the dense reduction
// buffer are never live together, so they share storage; the buffer makes a 3D MIXED
// block 75 KB, two per CU, which is also what 80 VGPRs at six waves per SIMD allow.  The
// block takes the storage as dynamic LDS: with a static size above a third of the CU's
// LDS the compiler would conclude that six waves per SIMD cannot be resident and spend
// more registers, which would leave one block per CU.
template <int D, typename R>
struct StressLds {
  static constexpr int NT = TileGeo<D>::NT, RN = TileGeo<D>::RN;
  static constexpr int CH = NT;                             // points per chunk
  static constexpr int PW = 4 * D + D * D;                  // x fn, w table, stress
  static constexpr int PS = PW | 1;                         // odd payload stride
  // 3D: the gathers' polynomial coefficients follow the payloads (they share the room of
  // the dense reduction buffer, which is only used after the last chunk)
  static constexpr int NCF = D == 3 ? MonoGeo<3>::N : 0;
  static_assert((CH * PS * sizeof(R)) % 16 == 0, "coefficients in 16-byte rows");
  R u[RN * D];
  double bsum[16];
  union alignas(16) {   // the dense buffer is cleared in 16-byte rows
    R pt[CH * PS + NCF];
    R dense[RN * D * DenseRed<D>::KS];
  } x;
};

// A point's inputs to the stress scatter, loaded one chunk ahead so that the loads are in
// flight while the previous chunk is scattered (and, for the first chunk, while the node
// region is staged).  Interior: x, J^n, V0, mu V^n; for the Hessian x and the two
// coefficients dt^2 lam V0 (J^n)^2 and dt mu V^n formed at the particle staging.  Surface:
// x, k_r, dA (the cached F_r of the Hessian is loaded in the point phase: holding it
// across the scatter spills).
template <int D, typename R, int MODE>
struct StressIn {
  static constexpr int NV = D + 1 + D;
  R v[NV];
  int k = -1;            // point index (sorted order), -1: none
  bool interior = true;
};

template <int D, typename R, int MODE>
MPM_DEV void stress_fetch(const Dev<R>& d, int q, int ntot, int npi, int pb, int sb, bool visc, StressIn<D, R, MODE>& in) {
  in.k = -1;
  if (q >= ntot) return;
  const int N = d.np, S = d.ns;
  in.interior = q < npi;
  const int k = in.interior ? pb + q : sb + (q - npi);
  in.k = k;
  // every slot is written on both paths (constant indices), so that the array stays in
  // registers
  if (in.interior) {
#pragma unroll
    for (int a = 0; a < D; ++a) in.v[a] = d.px[a * N + k];
    if constexpr (MODE == TM_HESS) {
      in.v[D] = d.pHc[k];
      in.v[D + 1] = visc ? d.pHc[N + k] : R(0);
      in.v[D + 2] = R(0);
    } else {
      in.v[D] = d.pJ[k];
      in.v[D + 1] = d.pV0[k];
      in.v[D + 2] = visc ? d.pmu[k] * d.pVn[k] : R(0);
    }
#pragma unroll
    for (int a = 2; a < D; ++a) in.v[D + 1 + a] = R(0);
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) in.v[a] = d.ss[a * S + k];
    in.v[D] = d.sk[k];
#pragma unroll
    for (int a = 0; a < D; ++a) in.v[D + 1 + a] = d.sdA[a * S + k];
  }
}

// A thread's share of a tile's node region: thread t < RN holds region node t, all of its
// D components (each load instruction of a wave reads one component of 64 consecutive
// region nodes).  All of a thread's loads (u, z and the node's free flags) are issued
// before any is used; the constraint mask and the CG direction are applied when the node
// is written to LDS.
template <int D, typename R>
struct RegionPf {
  R uv[D], zv[D];
  int fr;   // free flags of the node; 0 outside the grid or past the region
};

// org: the tile's first cell (tile_origin).
template <int D, typename R>
MPM_DEV void region_fetch(const Dev<R>& d, const int* org, const R* u, const R* z, int mask_in,
                          RegionPf<D, R>& pf) {
  constexpr int RN = TileGeo<D>::RN;
  static_assert(RN <= TileGeo<D>::NT, "one region node per thread");
  const int t = threadIdx.x;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    pf.uv[a] = R(0);
    pf.zv[a] = R(0);
  }
  pf.fr = 0;
  if (t >= RN) return;
  int r[3];
  region_coords<D>(t, r);
  const int gnode = region_node_at<D>(org, r, d.n, d.nt);
  if (gnode < 0) return;
  pf.fr = mask_in ? d.gfree[gnode] : 0xff;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    pf.uv[a] = u[a * d.nn + gnode];
    if (z) pf.zv[a] = z[a * d.nn + gnode];
  }
}

template <int D, typename R>
MPM_DEV void region_commit(const RegionPf<D, R>& pf, bool has_z, R beta, R* su) {
  const int t = threadIdx.x;
  if (t >= TileGeo<D>::RN) return;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    R uv = pf.uv[a];
    if (has_z) uv = cg_dir(pf.zv[a], beta, uv);
    su[t * D + a] = ((pf.fr >> a) & 1) ? uv : R(0);
  }
}

// Variants of the stress tile kernel: the fluid (J term, viscosity, surface), the fluid with
// the J term alone in its interior points (no viscosity: divergence and s I only), and the
// fluid with solid particles.  Each is its own instantiation, so that no variant carries
// the registers of another's paths.
enum StressVar { SV_FLUID = 0, SV_SOLID = 1, SV_JONLY = 2 };

template <int D, typename R, int MODE, int VAR = SV_FLUID>
__global__ void MPM_TILE_KERNEL(TileGeo<D>::NT, TileOcc<R>::STRESS) k_tile_stress(Dev<R> d, TileLists tl, const R* u, R* tpart,
                                                                int mask_in, const int* done, int energy_slot,
                                                                PUpd<R> pu, R* fout) {
  constexpr int NT = TileGeo<D>::NT, RN = TileGeo<D>::RN;
  constexpr int CH = StressLds<D, R>::CH, PS = StressLds<D, R>::PS;
  extern __shared__ __align__(16) unsigned char stress_lds[];
  StressLds<D, R>& sm = *reinterpret_cast<StressLds<D, R>*>(stress_lds);
  if (done && *done) return;
  const int slot = xcd_slot(blockIdx.x, tl.xrun);
  if (slot >= tl.nctile) return;
  const int ct = tl.ctile_list[slot];
  const int S = d.ns;
  const int t = threadIdx.x;
  const R dt = d.dt;
  int org[3] = {0, 0, 0};
  tile_origin<D>(ct, d.nt, org);
  const int cb = ct * 64;
  constexpr bool SOL = VAR == SV_SOLID, ISO = VAR == SV_JONLY, SYM = VAR == SV_FLUID;
  // 3D, but for the J term alone (whose s I scatter is cheaper node by node): the scatter
  // accumulates coefficient sensitivities (lane_scatter_mono)
  constexpr bool MONO = D == 3 && !ISO;
  const bool surf = (d.term_mask & 2) && S > 0;
  const bool vol = (d.term_mask & 5) != 0;
  const bool visc = !ISO && (d.term_mask & 4) != 0;
  const int* rg = tl.ctile_rng + 6 * slot;
  const int pb = rg[0], pe = vol ? rg[1] : pb;
  const int sb = surf ? rg[2] : 0, se = surf ? rg[3] : 0;
  const int npi = pe - pb;
  const int ntot = npi + (se - sb);
  // first chunk's point inputs, issued together with the node staging below
  StressIn<D, R, MODE> in;
  if (t < CH) stress_fetch<D, R, MODE>(d, t, ntot, npi, pb, sb, visc, in);
  const R beta = pu.beta();
  // the node region, the lanes' cell ranges: every load is issued before the region is
  // written to LDS, so that the block waits for one round trip
  RegionPf<D, R> pf;
  region_fetch<D, R>(d, org, u, pu.z, mask_in, pf);
  int lcell, lk0, lk1;
  lane_map<D>(t, lcell, lk0, lk1);
  const LaneDw<R> ldw0(lk0), ldw1(lk1);
  const bool lane_on = t < 64 * TileGeo<D>::LPC;
  int cpb = 0, cpe = 0, csb = 0, cse = 0;
  if (lane_on) {
    if (vol) { cpb = d.p_start[cb + lcell] - pb; cpe = d.p_start[cb + lcell + 1] - pb; }
    if (surf) { csb = d.s_start[cb + lcell] - sb + npi; cse = d.s_start[cb + lcell + 1] - sb + npi; }
  }
  region_commit<D, R>(pf, pu.z != nullptr, beta, sm.u);
  LaneAcc<D, R, D> acc;
  acc.zero();
  double e = 0;
  R* cf = sm.x.pt + CH * PS;
  __syncthreads();
  if constexpr (D == 3) {
    mono_build<R, 3>(sm.u, cf);
    __syncthreads();
  }
  for (int q0 = 0; q0 < ntot; q0 += CH) {
    // ---- point phase: weights, gradient of u, stress ----
    if (t < CH && in.k >= 0) {
      const bool interior = in.interior;
      R f[D];
      int lc[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < D; ++a) {
        R xs = in.v[a] * d.fn;
        R cf = floor(xs);
        f[a] = xs - cf;
        int l = (int)cf - org[a];
        lc[a] = l < 0 ? 0 : (l > TileGeo<D>::E - 1 ? TileGeo<D>::E - 1 : l);   // clamped points only
      }
      R w[D][3], dw[D][3];
      weight_table<D, R>(f, d.fn, w, dw);
      // the fluid's J term alone (no viscosity, no solids) needs only the divergence, and
      // its stress is s I: one payload value instead of D x D
      const bool jonly = ISO && interior;
      R G[D][D], val[D];
      R trj = 0;
      if constexpr (D == 3) {
        if (jonly) trj = mono_div<R>(cf, lc, f[0], f[1], d.fn, w[2], dw[2]);
        else mono_grad<R, 3>(cf, lc, f[0], f[1], d.fn, w[2], dw[2], G, val);
      } else {
        if (jonly) trj = region_div<D, R>(sm.u, lc, w, dw);
        else region_grad<D, R, D>(sm.u, lc, w, dw, G, val);
      }
      R Sq[D][D];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) Sq[a][b] = 0;
      if (SOL && interior && d.pSol[in.k] != R(0)) {
        // a solid particle: the fixed-corotated term in place of pressure and viscosity
        if (d.term_mask & 1) {
          const R es = solid_stress<D, R, MODE>(d, in.k, G, dt, fout, Sq);
          if (MODE == TM_ENERGY) e += (double)es;
        }
      } else if (interior) {
        R tr = 0;
        if (jonly) {
          tr = trj;
        } else {
#pragma unroll
          for (int a = 0; a < D; ++a) tr += G[a][a];
        }
        const R Jn = in.v[D], V0 = in.v[D + 1];
        if (d.term_mask & 1) {
          R s;
          if (MODE == TM_HESS) {
            s = in.v[D] * tr;                  // (dt^2 lam V0 (J^n)^2) tr
          } else {
            R Jm1 = (R(1) + dt * tr) * Jn - R(1);
            if (MODE == TM_ENERGY) e += (double)(R(0.5) * d.lam * Jm1 * Jm1 * V0);
            s = dt * d.lam * V0 * Jn * Jm1;
          }
#pragma unroll
          for (int a = 0; a < D; ++a) Sq[a][a] += s;
        }
        if (visc) {
          const R cV = MODE == TM_HESS ? in.v[D + 1] : dt * in.v[D + 2];
          R ee = 0;
#pragma unroll
          for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) {
              R eps = R(0.5) * (G[a][b] + G[b][a]);
              Sq[a][b] += cV * eps;
              ee += eps * eps;
            }
          if (MODE == TM_ENERGY) e += (double)(R(0.5) * cV * ee);
        }
      } else {
        R Nv[D], F[D][D];
        const R kr = in.v[D];
#pragma unroll
        for (int a = 0; a < D; ++a) Nv[a] = in.v[D + 1 + a];
        if constexpr (MODE == TM_HESS) {
#pragma unroll
          for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) F[a][b] = d.sF[(a * D + b) * d.ns + in.k];
        } else {
#pragma unroll
          for (int a = 0; a < D; ++a) {
#pragma unroll
            for (int b = 0; b < D; ++b) F[a][b] = dt * G[a][b];
            F[a][a] += R(1);
          }
          // the surface linearization point of a Hessian at this velocity
          if (fout) {
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
              for (int b = 0; b < D; ++b) fout[(a * D + b) * d.ns + in.k] = F[a][b];
          }
        }
        R Q[D][D];
        R an = surface_q<D, R>(F, Nv, MODE == TM_HESS, G, dt, d.exact, Q);
        if (MODE == TM_ENERGY) e += (double)(kr * an);
        const R sc = dt * kr;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) Sq[a][b] = sc * Q[a][b];
      }
      R* P = &sm.x.pt[t * PS];
      // MONO: x, y, fn wz, dwz and the stress at SO (lane_scatter_mono); else X = x fn (the
      // lanes form their derivatives from it), the weight table and the stress at 4 D
      constexpr int SO = MONO ? 8 : 4 * D;
      if constexpr (MONO) {
        P[0] = f[0];
        P[1] = f[1];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          P[2 + kk] = d.fn * w[2][kk];
          P[5 + kk] = dw[2][kk];
        }
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          P[a] = f[a] * d.fn;
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) P[D + a * 3 + kk] = w[a][kk];
        }
      }
      if (jonly) {
        P[SO] = Sq[0][0];
      } else if (SYM && interior && !MONO) {
        // the fluid's interior stress s I + cV sym(G) is symmetric: its upper triangle
#pragma unroll
        for (int a = 0, k = 0; a < D; ++a)
#pragma unroll
          for (int b = a; b < D; ++b, ++k) P[SO + k] = Sq[a][b];
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) P[SO + a * D + b] = Sq[a][b];
      }
    }
    __syncthreads();
    // next chunk's inputs, if there is one: in flight during this chunk's scatter
    if (q0 + CH < ntot && t < CH) stress_fetch<D, R, MODE>(d, q0 + CH + t, ntot, npi, pb, sb, visc, in);
    // ---- scatter phase: the lane's cell points inside this chunk ----
    if constexpr (MONO) {
      // lane (component a = lk0, plane kz = lk1): the a row of the stress
      const int lo = q0, hi = min(q0 + CH, ntot);
      const int a = lk0, kz = lk1;
      for (int pass = 0; pass < 2 && lane_on; ++pass) {
        const int b0 = max(pass == 0 ? cpb : csb, lo), b1 = min(pass == 0 ? cpe : cse, hi);
        for (int qq = b0; qq < b1; ++qq) {
          const R* P = &sm.x.pt[(qq - q0) * PS];
          const R* Sa = P + 8 + 3 * a;
          lane_scatter_mono<R>(P[0], P[1], P[2 + kz], P[5 + kz], Sa[0], Sa[1], Sa[2], acc.v);
        }
      }
    } else if (lane_on) {
      int lo = q0, hi = min(q0 + CH, ntot);
      for (int pass = 0; pass < 2; ++pass) {
        int b0 = max(pass == 0 ? cpb : csb, lo), b1 = min(pass == 0 ? cpe : cse, hi);
        if (ISO && pass == 0) {
          // interior points with the J term alone: s I
          for (int qq = b0; qq < b1; ++qq) {
            const R* P = &sm.x.pt[(qq - q0) * PS];
            lane_scatter_iso<D, R>(P, P + D, d.fn, lk0, lk1, ldw0, ldw1, P[4 * D], acc.v);
          }
          continue;
        }
        if (SYM && pass == 0) {
          // interior points of the fluid: the stress from its upper triangle
          for (int qq = b0; qq < b1; ++qq) {
            const R* P = &sm.x.pt[(qq - q0) * PS];
            R Sq[D][D];
#pragma unroll
            for (int a = 0, k = 0; a < D; ++a)
#pragma unroll
              for (int b = a; b < D; ++b, ++k) Sq[a][b] = Sq[b][a] = P[4 * D + k];
            lane_scatter_grad<D, R>(P, P + D, d.fn, lk0, lk1, ldw0, ldw1, Sq, acc.v);
          }
          continue;
        }
        for (int qq = b0; qq < b1; ++qq) {
          const R* P = &sm.x.pt[(qq - q0) * PS];
          R Sq[D][D];
#pragma unroll
          for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) Sq[a][b] = P[4 * D + a * D + b];
          lane_scatter_grad<D, R>(P, P + D, d.fn, lk0, lk1, ldw0, ldw1, Sq, acc.v);
        }
      }
    }
    __syncthreads();
  }
  // ---- reduce onto the region and write the tile partial ----
  R* dst = tpart + (size_t)slot * RN * D;
  auto wr = [&](int rn, int f, R v) { dst[rn * D + f] = v; };
  reduce_region_dense<D, R, D, decltype(wr)&, MONO>(acc, sm.x.dense, lcell, lk0, lk1, lane_on, wr);
  if (MODE == TM_ENERGY && energy_slot >= 0) {
    double bs = block_sum(e, sm.bsum);
    if (t == 0) d.part[energy_slot * kPartSlot + slot] = bs;
  }
}

// Linearization point of the surface term: F_r = I + dt grad v_lin(s_r), cached per sample.
template <int D, typename R>
__global__ void k_surface_F(Dev<R> d, const R* vlin) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int S = d.ns;
  if (r >= S) return;
  R x[D];
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = d.ss[a * S + r];
  Stencil<D, R> st; bool bad = false;
  make_stencil<D, R>(x, d.n, d.fn, st, &bad);
  R G[D][D];
  gather_grad<D, R>(d, st, vlin, false, G);
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) d.sF[(a * D + b) * S + r] = (a == b ? R(1) : R(0)) + d.dt * G[a][b];
}

// Linearization point of the solid particles: cof F_p of F_p = (I + dt grad v_lin(x_p)) F^n_p,
// cached after the surface part.
template <int D, typename R>
__global__ void k_solid_lin(Dev<R> d, const R* vlin) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = d.np;
  if (k >= N || d.pSol[k] == R(0)) return;
  R x[D];
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = d.px[a * N + k];
  Stencil<D, R> st; bool bad = false;
  make_stencil<D, R>(x, d.n, d.fn, st, &bad);
  R G[D][D];
  gather_grad<D, R>(d, st, vlin, false, G);
  R F[D][D], C[D][D];
  solid_F<D, R>(d, k, G, d.dt, F);
  cofactor_of<D, R>(F, C);
  R* cache = d.sF + (size_t)D * D * d.ns;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) cache[(a * D + b) * N + k] = C[a][b];
}

// ======================================================================================
// Heat operator scatter: interior points carry q_p = K V^n grad T_p (vector), surface
// samples c_r = h |dA_r| T(s_r) (scalar); contribution c N_i + q . grad N_i.
// ======================================================================================
template <int D, typename R>
struct HeatLds {
  static constexpr int NT = TileGeo<D>::NT, RN = TileGeo<D>::RN;
  static constexpr int CH = NT;                             // points per chunk
  static constexpr int PW = 4 * D + 1 + D;    // x fn, w table, c, q
  static constexpr int PS = PW | 1;           // odd payload stride (distinct banks per cell)
  // 3D: the gather's polynomial coefficients follow the payloads
  static constexpr int NCF = D == 3 ? MonoGeo<1>::N : 0;
  static_assert((CH * PS * sizeof(R)) % 16 == 0 || NCF == 0, "coefficients in 16-byte rows");
  R u[RN];
  union alignas(16) {   // the dense buffer is cleared in 16-byte rows
    R pt[CH * PS + NCF];
    R dense[RN * DenseRed<D>::KS];
  } x;
};

template <int D, typename R>
__global__ void MPM_TILE_KERNEL(TileGeo<D>::NT, TileOcc<R>::HEAT) k_tile_heat(Dev<R> d, TileLists tl, const R* T, R* tpart,
                                                              const int* done, PUpd<R> pu) {
  constexpr int NT = TileGeo<D>::NT, RN = TileGeo<D>::RN, PS = HeatLds<D, R>::PS, CH = HeatLds<D, R>::CH;
  __shared__ HeatLds<D, R> sm;
  if (done && *done) return;
  const int slot = xcd_slot(blockIdx.x, tl.xrun);
  if (slot >= tl.nctile) return;
  const int ct = tl.ctile_list[slot];
  const int N = d.np, S = d.ns;
  const int t = threadIdx.x;
  int org[3] = {0, 0, 0};
  tile_origin<D>(ct, d.nt, org);
  const R beta = pu.beta();
  // the region's values and the lanes' cell ranges are all loaded before the region is
  // written to LDS (one round trip); the region has fewer nodes than the block threads
  static_assert(RN <= NT, "one region node per thread");
  R tv = R(0), zv = R(0);
  int gnode = -1;
  if (t < RN) {
    int r[3];
    region_coords<D>(t, r);
    gnode = region_node_at<D>(org, r, d.n, d.nt);
    if (gnode >= 0) {
      tv = T[gnode];
      if (pu.z) zv = pu.z[gnode];
    }
  }
  const int cb = ct * 64;
  const int* rg = tl.ctile_rng + 6 * slot;
  const int pb = rg[0], pe = rg[1];
  const int sb = S ? rg[2] : 0, se = S ? rg[3] : 0;
  const int npi = pe - pb, ntot = npi + (se - sb);
  // 3D: the scatter accumulates coefficient sensitivities (lane_scatter_mono_g), one lane
  // per (cell, z plane), 192 lanes; 2D: lanes (cell, k0) over the nodes
  constexpr bool HM = D == 3;
  int lcell, lk0, lk1;
  lane_map<D>(t, lcell, lk0, lk1);
  if constexpr (HM) {
    lcell = t / 3;
    lk0 = 0;
    lk1 = t % 3;
  }
  const LaneDw<R> ldw0(lk0), ldw1(lk1);
  const bool lane_on = t < 64 * (HM ? 3 : TileGeo<D>::LPC);
  int cpb = 0, cpe = 0, csb = 0, cse = 0;
  if (lane_on) {
    cpb = d.p_start[cb + lcell] - pb; cpe = d.p_start[cb + lcell + 1] - pb;
    if (S) { csb = d.s_start[cb + lcell] - sb + npi; cse = d.s_start[cb + lcell + 1] - sb + npi; }
  }
  if (t < RN) sm.u[t] = gnode >= 0 ? (pu.z ? cg_dir(zv, beta, tv) : tv) : R(0);
  std::conditional_t<HM, LaneAcc<3, R, 3>, LaneAcc<D, R, 1>> acc;
  acc.zero();
  R* cf = sm.x.pt + CH * PS;
  __syncthreads();
  if constexpr (D == 3) {
    mono_build<R, 1>(sm.u, cf);
    __syncthreads();
  }
  for (int q0 = 0; q0 < ntot; q0 += CH) {
    int q = q0 + t;
    if (t < CH && q < ntot) {
      bool interior = q < npi;
      int k = interior ? pb + q : sb + (q - npi);
      R f[D];
      int lc[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < D; ++a) {
        R xs = (interior ? d.px[a * N + k] : d.ss[a * S + k]) * d.fn;
        R cf = floor(xs);
        f[a] = xs - cf;
        int l = (int)cf - org[a];
        lc[a] = l < 0 ? 0 : (l > TileGeo<D>::E - 1 ? TileGeo<D>::E - 1 : l);
      }
      R w[D][3], dw[D][3];
      weight_table<D, R>(f, d.fn, w, dw);
      R G[1][D], val[1];
      if constexpr (D == 3) mono_grad<R, 1>(cf, lc, f[0], f[1], d.fn, w[2], dw[2], G, val);
      else region_grad<D, R, 1>(sm.u, lc, w, dw, G, val);
      R* P = &sm.x.pt[t * PS];
      // 3D: x, y, fn wz, dwz, wz, then c and q at CO; 2D: X = x fn (the lanes form their
      // derivatives from it), the weight table, then c and q
      constexpr int CO = HM ? 11 : 4 * D;
      if constexpr (HM) {
        P[0] = f[0];
        P[1] = f[1];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          P[2 + kk] = d.fn * w[2][kk];
          P[5 + kk] = dw[2][kk];
          P[8 + kk] = w[2][kk];
        }
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          P[a] = f[a] * d.fn;
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) P[D + a * 3 + kk] = w[a][kk];
        }
      }
      if (interior) {
        R c = d.K * d.pVn[k];
        P[CO] = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) P[CO + 1 + a] = c * G[0][a];
      } else {
        R area = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) area += d.sdA[a * S + k] * d.sdA[a * S + k];
        P[CO] = d.h * sqrt(area) * val[0];
#pragma unroll
        for (int a = 0; a < D; ++a) P[CO + 1 + a] = 0;
      }
    }
    __syncthreads();
    if (lane_on) {
      int lo = q0, hi = min(q0 + CH, ntot);
      for (int pass = 0; pass < 2; ++pass) {
        int b0 = max(pass == 0 ? cpb : csb, lo), b1 = min(pass == 0 ? cpe : cse, hi);
        for (int qq = b0; qq < b1; ++qq) {
          const R* P = &sm.x.pt[(qq - q0) * PS];
          if constexpr (HM) {
            // c N + q . grad N: gA = q_0 fn wz, gB = q_1 fn wz, gC = c wz + q_2 dwz
            const R fw = P[2 + lk1], dwz = P[5 + lk1], wz = P[8 + lk1];
            lane_scatter_mono_g<R>(P[0], P[1], P[12] * fw, P[13] * fw, fma_r(P[11], wz, P[14] * dwz), acc.v);
          } else {
            lane_scatter_heat<D, R>(P, P + D, d.fn, lk0, lk1, ldw0, ldw1, P[4 * D], P + 4 * D + 1, acc.v);
          }
        }
      }
    }
    __syncthreads();
  }
  R* dst = tpart + (size_t)slot * RN;
  auto wr = [&](int rn, int, R v) { dst[rn] = v; };
  reduce_region_dense<D, R, 1, decltype(wr)&, HM>(acc, sm.x.dense, lcell, lk0, lk1, lane_on, wr);
}

// ======================================================================================
// P2G scatter (Section 4.2) with the set-up sums.  Fields per node:
//   0 m, 1..D mv, D+1 W, D+2 WT, D+3 E, D+4 ET, D+5..2D+4 Newton diagonal terms,
//   2D+5 heat diagonal terms, 2D+6 heat right-side terms.   NF = 2D + 7.
// Per point: m~ and the APIC momentum, or unsplit m with T, grad T (interior), or the
// parent's temperature (split members); contributions N (c + B rel) with rel = x_i - x_q,
// plus quadratic terms of grad N for the diagonals.
// ======================================================================================
template <int D> struct P2GF {
  static constexpr int NF = 2 * D + 7;
  static constexpr int M = 0, MV = 1, WT = D + 1, E = D + 2, ET = D + 3, W = D + 4, DG = D + 5, HD = 2 * D + 5,
                       HR = 2 * D + 6;
  // The fields go in two groups, each transferred by its own workgroup of one launch:
  // group 0 (fields [0, G1)) needs the weights only; group 1 (fields [G1, NF)) the weight
  // gradients for all but W, which joins it because, like the gradient terms, it comes
  // from the interior particles alone (with 7 fields per reduction round in FP32, both
  // groups then reduce in one round).  Payload per point of group 0: m~, m~ v, m~ A, c_W
  // (unused), c_WT, c_E, c_ET, m grad T; of group 1: cJ, cV, cK (|grad N|^2 heat term), cR
  // (N^2 Robin term), cS (N heat right side), c_W.
  static constexpr int G1 = D + 4;
  static constexpr int PL0 = 1 + D + D * D + 4 + D, PL1 = 6;
  static constexpr int PW0 = D + 3 * D + PL0;        // f, w table, payload
  static constexpr int PW1 = D + 6 * D + PL1;        // f, w and dw tables, payload
  static constexpr int PW = PW0 > PW1 ? PW0 : PW1;
};

// LDS of the P2G tile kernel.  The payload stride is odd, so that the points that the
// cells of a wave read at one time fall in distinct banks.
template <int D, typename R>
struct P2GLds {
  static constexpr int NT = TileGeo<D>::NT, RN = TileGeo<D>::RN;
  static constexpr int CH = NT / 2;                              // points per chunk
  static constexpr int FC = 7;                                   // fields per reduction round
  static constexpr int PS = P2GF<D>::PW | 1;                     // payload stride
  union {
    R pay[CH * PS];
    struct {
      R cellpart[64 * 27 * FC];   // the region sums go straight to the tile partial
    } red;
  } x;
};

// Weights of the lane's three nodes (the weight factor of lane_nodes alone).
template <int D, typename R>
MPM_DEV void lane_weights(const R* W, int k0, int k1, R (&wn)[3]) {
  if constexpr (D == 3) {
    R ga = W[0 * 3 + k0] * W[1 * 3 + k1];
#pragma unroll
    for (int k = 0; k < 3; ++k) wn[k] = ga * W[2 * 3 + k];
  } else {
    R wx = W[k0];
#pragma unroll
    for (int k = 0; k < 3; ++k) wn[k] = wx * W[3 + k];
  }
}

// One field group G of the P2G transfer for cell tile ti (position in the cell-tile list).
template <int D, typename R, int G>
MPM_DEV void p2g_group(const Dev<R>& d, const TileLists& tl, int ti, R* tpart, P2GLds<D, R>& sm) {
  constexpr int NT = TileGeo<D>::NT, RN = TileGeo<D>::RN;
  using FI = P2GF<D>;
  constexpr int F0 = G == 0 ? 0 : FI::G1, NFG = G == 0 ? FI::G1 : FI::NF - FI::G1;
  constexpr int PS = P2GLds<D, R>::PS, CH = P2GLds<D, R>::CH, FC = P2GLds<D, R>::FC;
  const int ct = tl.ctile_list[ti];
  const int N = d.np, S = d.ns;
  const int t = threadIdx.x;
  const R dt = d.dt;
  const int cb = ct * 64;
  const int pb = d.p_start[cb], pe = d.p_start[cb + 64];
  const int sb = S ? d.s_start[cb] : 0, se = S ? d.s_start[cb + 64] : 0;
  const int bb = S ? d.b_start[cb] : 0, be = S ? d.b_start[cb + 64] : 0;
  const int n1 = pe - pb, n2 = n1 + (se - sb);
  // group 1 has nothing from balance particles (all of its payload terms vanish for them)
  const int ntot = G == 0 ? n2 + (be - bb) : n2;
  constexpr int NPASS = G == 0 ? 3 : 2;
  int lcell, lk0, lk1;
  lane_map<D>(t, lcell, lk0, lk1);
  const bool lane_on = t < 64 * TileGeo<D>::LPC;
  int rb[3] = {0, 0, 0}, re[3] = {0, 0, 0};
  if (lane_on) {
    rb[0] = d.p_start[cb + lcell] - pb; re[0] = d.p_start[cb + lcell + 1] - pb;
    if (S) {
      rb[1] = d.s_start[cb + lcell] - sb + n1; re[1] = d.s_start[cb + lcell + 1] - sb + n1;
      rb[2] = d.b_start[cb + lcell] - bb + n2; re[2] = d.b_start[cb + lcell + 1] - bb + n2;
    }
  }
  const bool useJ = d.term_mask & 1, useV = d.term_mask & 4;
  LaneAcc<D, R, NFG> acc;
  acc.zero();
  for (int q0 = 0; q0 < ntot; q0 += CH) {
    int q = q0 + t;
    if (t < CH && q < ntot) {
      R* P = &sm.x.pay[t * PS];
      int type = q < n1 ? 0 : (q < n2 ? 1 : 2);
      int k, p;
      R x[D];
      if (type == 0) { k = pb + q; p = k; for (int a = 0; a < D; ++a) x[a] = d.px[a * N + k]; }
      else if (type == 1) { k = sb + (q - n1); p = d.spar[k]; for (int a = 0; a < D; ++a) x[a] = d.ss[a * S + k]; }
      else { k = bb + (q - n2); p = d.spar[d.b_src[k]]; for (int a = 0; a < D; ++a) x[a] = d.bx[a * S + k]; }
      R fq[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        R xs = x[a] * d.fn;
        fq[a] = xs - floor(xs);
        P[a] = fq[a];
      }
      {
        R w[D][3], dw[D][3];
        weight_table<D, R>(fq, d.fn, w, dw);
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) {
            P[D + a * 3 + kk] = w[a][kk];
            if (G == 1) P[4 * D + a * 3 + kk] = dw[a][kk];
          }
      }
      if constexpr (G == 0) {
        R* Q = P + 4 * D;                   // m~, m~ v, m~ A
        R mt = d.pmt[p];
        Q[0] = mt;
#pragma unroll
        for (int a = 0; a < D; ++a) Q[1 + a] = mt * d.pv[a * N + p];
#pragma unroll
        for (int a = 0; a < D * D; ++a) Q[1 + D + a] = mt * d.pA[a * N + p];
        R* Z = Q + 1 + D + D * D;           // c_W, c_WT, c_E, c_ET
        R* bW = Z + 4;                      // m grad T
        if (type == 0) {
          R mp = d.pm[k];
          Z[0] = mp; Z[1] = mp * d.pT[k]; Z[2] = 0; Z[3] = 0;
#pragma unroll
          for (int a = 0; a < D; ++a) bW[a] = mp * d.pgT[a * N + k];
        } else {
          Z[0] = 0; Z[1] = 0; Z[2] = mt; Z[3] = mt * d.pT[p];
#pragma unroll
          for (int a = 0; a < D; ++a) bW[a] = 0;
        }
      } else {
        R* H = P + 7 * D;                   // cJ, cV, cK, cR, cS
        if (type == 0) {
          R Jn = d.pJ[k], Vn = d.pVn[k];
          const bool solid = d.solids && d.pSol[k] != R(0);   // no fluid pressure in a solid
          H[0] = useJ && !solid ? dt * dt * d.lam * d.pV0[k] * Jn * Jn : R(0);
          H[1] = useV ? dt * d.pmu[k] * Vn : R(0);
          H[2] = d.K * Vn;
          H[3] = 0;
          H[4] = d.H * Vn;
          H[5] = d.pm[k];
        } else {
          R area = 0;
#pragma unroll
          for (int a = 0; a < D; ++a) area += d.sdA[a * S + k] * d.sdA[a * S + k];
          area = sqrt(area);
          H[0] = 0; H[1] = 0; H[2] = 0;
          H[3] = d.h * area;
          H[4] = (d.h * d.T_amb + d.b) * area;
          H[5] = 0;
        }
      }
    }
    __syncthreads();
    if (lane_on) {
      int lo = q0, hi = min(q0 + CH, ntot);
      // pass 0: interior particles, 1: surface samples, 2: balance points.  Each type
      // leaves some fields at zero (interior: E, ET and the Robin term; samples and balance
      // points: W, WT and the Hessian diagonal), so the passes skip them.
#pragma unroll
      for (int pass = 0; pass < NPASS; ++pass) {
        const bool interior = pass == 0;
        int b0 = max(rb[pass], lo), b1 = min(re[pass], hi);
        for (int qq = b0; qq < b1; ++qq) {
          const R* P = &sm.x.pay[(qq - q0) * PS];
          if constexpr (G == 0) {
            R f[D];
#pragma unroll
            for (int a = 0; a < D; ++a) f[a] = P[a];
            R wn[3];
            lane_weights<D, R>(P + D, lk0, lk1, wn);
            const R* Q = P + 4 * D;
            const R* Z = Q + 1 + D + D * D;
            const R* bW = Z + 4;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              const R w = wn[k];
              int kk[3] = {lk0, D == 3 ? lk1 : k, D == 3 ? k : 0};
              R rel[D];
#pragma unroll
              for (int a = 0; a < D; ++a) rel[a] = (R(kk[a]) - R(0.5) - f[a]) * d.dx;
              acc.v[k][FI::M] += w * Q[0];
#pragma unroll
              for (int a = 0; a < D; ++a) {
                R s = Q[1 + a];
#pragma unroll
                for (int b = 0; b < D; ++b) s += Q[1 + D + a * D + b] * rel[b];
                acc.v[k][FI::MV + a] += w * s;
              }
              if (interior) {
                R sw = Z[1];
#pragma unroll
                for (int a = 0; a < D; ++a) sw += bW[a] * rel[a];
                acc.v[k][FI::WT] += w * sw;
              } else {
                acc.v[k][FI::E] += w * Z[2];
                acc.v[k][FI::ET] += w * Z[3];
              }
            }
          } else {
            const R* H = P + 7 * D;
            if (interior) {
              R wn[3], gn[3][D];
              lane_nodes<D, R>(P + D, P + 4 * D, lk0, lk1, wn, gn);
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                const R* g = gn[k];
                const R w = wn[k];
                R g2 = 0;
#pragma unroll
                for (int a = 0; a < D; ++a) g2 += g[a] * g[a];
#pragma unroll
                for (int a = 0; a < D; ++a)
                  acc.v[k][FI::DG - F0 + a] += H[0] * g[a] * g[a] + H[1] * (R(0.5) * g2 + R(0.5) * g[a] * g[a]);
                acc.v[k][FI::HD - F0] += H[2] * g2;
                acc.v[k][FI::HR - F0] += H[4] * w;
                acc.v[k][FI::W - F0] += w * H[5];
              }
            } else {
              R wn[3];
              lane_weights<D, R>(P + D, lk0, lk1, wn);
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                acc.v[k][FI::HD - F0] += H[3] * wn[k] * wn[k];
                acc.v[k][FI::HR - F0] += H[4] * wn[k];
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }
  // field rounds of FC onto the region, written to the tile partial
#pragma unroll
  for (int f0 = 0; f0 < NFG; f0 += FC) {
    reduce_cells_to_region_out<D, R, NFG, FC>(acc, f0, sm.x.red.cellpart, lcell, lk0, lk1, lane_on,
                                              [&](int rn, int f, R v) {
                                                tpart[((size_t)ti * RN + rn) * FI::NF + F0 + f0 + f] = v;
                                              });
  }
}

// P2G scatter, two workgroups per cell tile (one per field group).  Workgroups are handed
// to the XCDs in turn, so ids 16j + i and 16j + 8 + i (i < 8), which share an XCD and its
// L2, take the two groups of cell tile t0 + 8j + i.  The count of active cell tiles is
// read on the device (*nct), so that the launch can be sized before the host knows it:
// workgroups past it return at once, and a second launch with t0 > 0 covers the rest.
template <int D, typename R>
__global__ void MPM_TILE_KERNEL(TileGeo<D>::NT, TileOcc<R>::P2G) k_tile_p2g(Dev<R> d, TileLists tl, R* tpart,
                                                             const int* nct, int t0) {
  __shared__ P2GLds<D, R> sm;
  const int b = blockIdx.x;
  const int ti = t0 + (b >> 4) * 8 + (b & 7);
  if (ti >= *nct) return;
  if (b & 8) p2g_group<D, R, 1>(d, tl, ti, tpart, sm);
  else p2g_group<D, R, 0>(d, tl, ti, tpart, sm);
}

// ======================================================================================
// G2P with merge (Section 5), one workgroup per cell tile: v^ (and T^) staged on the
// tile's node region, one lane per interior particle, stencil sums by sum factorization.
// The particle's own share is m~ [v(x_p), sum_i N_i v^_i (x_i - x_p)^T]; the split members'
// shares come from k_g2p_split.  The state is written back in cell order.
// ======================================================================================
// sum_k N_k u_a (k_b) over the 3^D stencil: first moments of the staged field, from which
// sum_i N_i u_a (x_i - x_p)_b = dx [mom_ab - (f_b + 1/2) val_a] (x_i - x_p = (k - 1/2 - f) dx).
template <int D, typename R, int NC>
MPM_DEV void region_moments(const R* u, const int* lc, const R (&w)[D][3], R (&val)[NC], R (&mom)[NC][D]) {
  constexpr int RE = TileGeo<D>::RE;
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    val[a] = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) mom[a][b] = 0;
  }
  if constexpr (D == 3) {
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) {
      R V[NC], M0[NC], M1[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) { V[a] = 0; M0[a] = 0; M1[a] = 0; }
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) {
        int base = lc[0] + RE * ((lc[1] + k1) + RE * (lc[2] + k2));
#pragma unroll
        for (int a = 0; a < NC; ++a) {
          R u0 = u[(base + 0) * NC + a], u1 = u[(base + 1) * NC + a], u2 = u[(base + 2) * NC + a];
          R s = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
          R s1 = u1 * w[0][1] + R(2) * u2 * w[0][2];          // sum_k0 u w0 k0
          V[a] += s * w[1][k1];
          M0[a] += s1 * w[1][k1];
          M1[a] += s * w[1][k1] * R(k1);
        }
      }
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        val[a] += V[a] * w[2][k2];
        mom[a][0] += M0[a] * w[2][k2];
        mom[a][1] += M1[a] * w[2][k2];
        mom[a][2] += V[a] * w[2][k2] * R(k2);
      }
    }
  } else {
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      int base = lc[0] + RE * (lc[1] + k1);
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        R u0 = u[(base + 0) * NC + a], u1 = u[(base + 1) * NC + a], u2 = u[(base + 2) * NC + a];
        R s = u0 * w[0][0] + u1 * w[0][1] + u2 * w[0][2];
        R s1 = u1 * w[0][1] + R(2) * u2 * w[0][2];
        val[a] += s * w[1][k1];
        mom[a][0] += s1 * w[1][k1];
        mom[a][1] += s * w[1][k1] * R(k1);
      }
    }
  }
}

template <int D, typename R>
struct G2PLds {
  static constexpr int RN = TileGeo<D>::RN;
  R u[RN * D];
  R T[RN];
};

template <int D, typename R, bool SOL = false>
__global__ void __launch_bounds__(256) k_tile_g2p(Dev<R> d, TileLists tl, const R* vh, const R* Th, R* x, R* v,
                                                  R* A, R* J, R* V0, R* m, R* T, R* gT, R* Fout) {
  constexpr int NT = 256, RN = TileGeo<D>::RN;
  __shared__ G2PLds<D, R> sm;
  const int ct = tl.ctile_list[blockIdx.x];
  const int* rg = tl.ctile_rng + 6 * blockIdx.x;
  const int pb = rg[0], pe = rg[1];
  const int N = d.np, S = d.ns, nn = d.nn;
  const int t = threadIdx.x;
  int org[3] = {0, 0, 0};
  tile_origin<D>(ct, d.nt, org);
  for (int rn = t; rn < RN; rn += NT) {
    int r[3];
    region_coords<D>(rn, r);
    int gnode = region_node_at<D>(org, r, d.n, d.nt);
#pragma unroll
    for (int a = 0; a < D; ++a) sm.u[rn * D + a] = gnode >= 0 ? vh[a * nn + gnode] : R(0);
    sm.T[rn] = (gnode >= 0 && Th) ? Th[gnode] : R(0);
  }
  __syncthreads();
  for (int k = pb + t; k < pe; k += NT) {
    R xp[D], f[D];
    int lc[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      xp[a] = d.px[a * N + k];
      R xs = xp[a] * d.fn;
      R cf = floor(xs);
      f[a] = xs - cf;
      int l = (int)cf - org[a];
      lc[a] = l < 0 ? 0 : (l > TileGeo<D>::E - 1 ? TileGeo<D>::E - 1 : l);
    }
    R w[D][3], dw[D][3];
    weight_table<D, R>(f, d.fn, w, dw);
    R G[D][D], val[D], mom[D][D];
    region_grad<D, R, D>(sm.u, lc, w, dw, G, val);
    region_moments<D, R, D>(sm.u, lc, w, val, mom);
    R div = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) div += G[a][a];
    const R mt = d.pmt[k], mp = d.pm[k];
    R mo[D], tt[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      mo[a] = mt * val[a];
#pragma unroll
      for (int b = 0; b < D; ++b) tt[a][b] = mt * d.dx * (mom[a][b] - (f[b] + R(0.5)) * val[a]);
    }
    for (int j = d.grp_start[k]; j < d.grp_start[k + 1]; ++j) {
      int r = d.grp[j];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        mo[a] += mt * d.sc[a * S + r];
#pragma unroll
        for (int b = 0; b < D; ++b) tt[a][b] += mt * d.sc[(D + a * D + b) * S + r];
      }
    }
    const R inv_m = R(1) / mp, cA = R(4) / (mp * d.dx * d.dx);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R va = mo[a] * inv_m;
      v[a * N + k] = va;
      x[a * N + k] = xp[a] + d.dt * va;
#pragma unroll
      for (int b = 0; b < D; ++b) A[(a * D + b) * N + k] = cA * tt[a][b];
    }
    R Jnew = (R(1) + d.dt * div) * d.pJ[k];
    V0[k] = d.pV0[k];
    m[k] = mp;
    R Tnew;
    if (Th) {
      R GT[1][D], vT[1];
      region_grad<D, R, 1>(sm.T, lc, w, dw, GT, vT);
      Tnew = vT[0];
#pragma unroll
      for (int a = 0; a < D; ++a) gT[a * N + k] = GT[0][a];
    } else {
      Tnew = d.pT[k];
#pragma unroll
      for (int a = 0; a < D; ++a) gT[a * N + k] = d.pgT[a * N + k];
    }
    T[k] = Tnew;
    if (SOL && Fout) {
      // solids: F <- (I + dt grad v^) F, J = det F; then the phase change at T_melt
      // (melting: J = 1, F = I; freezing: F = I, J = 1), decided in FP64
      R Fk[D][D];
      const bool was = d.pSol[k] != R(0);
      if (was) {
        solid_F<D, R>(d, k, G, d.dt, Fk);
        Jnew = det_of<D, R>(Fk);
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) Fk[a][b] = d.pF[(a * D + b) * N + k];
      }
      const bool now = (double)Tnew < d.T_melt;
      if (was != now) {
        Jnew = R(1);
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) Fk[a][b] = a == b ? R(1) : R(0);
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) Fout[(a * D + b) * N + k] = Fk[a][b];
    }
    J[k] = Jnew;
  }
}

// ======================================================================================
// Merge: for every node of the active node tiles, sum the region partials of the <= 2^d
// cell tiles that cover it (fixed order: cell tiles in lexicographic order).
// ======================================================================================

// Node kernels of the operators: one wave per node tile, kMergeTiles tiles per block.  The
// blocks go to the XCDs in runs of kMergeRun (xcd_slot): a cell tile's partial is read by
// the merges of its own node tile and of its neighbours, and the neighbours along x (and
// some along y) then take its lines from the same L2.  Blocks past the last tile only
// join the grid sums.
constexpr int kMergeTiles = 4;
constexpr int kMergeRun = 16;
inline int merge_grid(int ntiles) { return xcd_grid((ntiles + kMergeTiles - 1) / kMergeTiles, kMergeRun); }

// Stress merge: node-level terms.
//  NM_GRAD: out = P[acc + m (v^ - v^n) - dt m g]; with phi the blocks also sum the tile
//           energy partials (epart, nep entries) and the grid sums go to red: red[0] = Phi,
//           red[1..D] = sum m (v^ - v^n), red[D+1] = sum m (nodes with mass), red[D+2] =
//           |out|^2, red[D+3] = slope_g . u (u before the input update; 0 without slope_g),
//           red[D+4] = sum over free components of (|acc| + m |u| + m |v^n| + dt m |g|)^2,
//           the size of the terms a component of the gradient is formed from (its
//           round-off in the arithmetic of R is about eps_R times the square root).
//  NM_HESS: out = P[acc + alpha m w]; with cg the grid sum of w . out sets the CG step.
// The mode is a template argument: the Hessian form, launched once per CG iteration, then
// carries neither the registers nor the LDS of the gradient form's sums.
template <int D, typename R, int MODE>
__global__ void __launch_bounds__(64 * kMergeTiles) k_merge_stress(
    Dev<R> d, TileLists tl, int ntiles, const R* tpart, const R* u, R* out, double alpha, int mask_in,
    const int* done, const double* epart, int nep, double* npart, unsigned* ctr, double* red, double* phi2,
    CgScal* cg, PUpd<R> pu, const R* slope_g) {
  constexpr int RN = TileGeo<D>::RN;
  constexpr int NV = D + 5;
  constexpr int mode = MODE;
  __shared__ double sh[(MODE == NM_GRAD ? NV : 1) * 64 * kMergeTiles];
  if (done && *done) return;
  const int ti = xcd_slot(blockIdx.x, kMergeRun) * kMergeTiles + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double vals[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) vals[k] = 0;
  double dotv = 0;
  if (ti < ntiles) {
    const int tile = d.tile_list[ti];
    const int node = tile * kTileNodes + lane;
    const int nn = d.nn;
    MergeSrc<D> ms;
    merge_sources_tab<D>(ti, lane, tl.nbr, ms);
    R acc[D];
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] = 0;
    R val[1 << D][D];
#pragma unroll
    for (int j = 0; j < (1 << D); ++j) {
      const R* src = tpart + (size_t)(ms.slot[j] < 0 ? 0 : ms.slot[j]) * RN * D + ms.rn[j] * D;
#pragma unroll
      for (int a = 0; a < D; ++a) val[j][a] = ms.slot[j] >= 0 ? src[a] : R(0);
    }
#pragma unroll
    for (int j = 0; j < (1 << D); ++j)
#pragma unroll
      for (int a = 0; a < D; ++a) acc[a] += val[j][a];
    uint8_t fr = d.gfree[node];
    R m = d.gm[node];
    const bool dof = fr & 0x80;
    if (dof && mode == NM_GRAD) vals[D + 1] = (double)m;
    const R beta = pu.beta();
    // the node's loads before its stores (a store may alias a later load for the compiler)
    R uv[D], sgv[D], zv[D], vnv[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      uv[a] = u ? u[a * nn + node] : R(0);
      sgv[a] = slope_g ? slope_g[a * nn + node] : R(0);
      zv[a] = pu.z ? pu.z[a * nn + node] : R(0);
      vnv[a] = mode == NM_GRAD ? d.gvn[a * nn + node] : R(0);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      bool fa = (fr >> a) & 1;
      R ua = uv[a];
      if (slope_g) vals[D + 3] += (double)sgv[a] * (double)ua;
      if (pu.z) {
        ua = cg_dir(zv[a], beta, ua);
        pu.p[a * nn + node] = ua;
      }
      R o;
      if (mode == NM_GRAD) {
        R vn = vnv[a];
        o = acc[a] + m * (ua - vn) - d.dt * m * d.grav[a];
        if (dof) {
          double dv = (double)ua - (double)vn;
          vals[0] += 0.5 * (double)m * dv * dv - (double)d.dt * (double)m * (double)d.grav[a] * (double)ua;
          vals[1 + a] = (double)m * dv;
        }
        if (fa) {
          const double mag = fabs((double)acc[a]) + fabs((double)m) * (fabs((double)ua) + fabs((double)vn) +
                                                                      fabs((double)d.dt * (double)d.grav[a]));
          vals[D + 4] += mag * mag;
        }
      } else {
        R wa = (!mask_in || fa) ? ua : R(0);
        o = acc[a] + R(alpha) * m * wa;
        if (fa) dotv += (double)wa * (double)o;
      }
      o = fa ? o : R(0);
      out[a * nn + node] = o;
      vals[D + 2] += (double)o * (double)o;
    }
  }
  const bool want = (mode == NM_GRAD && red) || (mode == NM_HESS && cg);
  if (!want) return;
  if (mode == NM_GRAD) {
    if (epart) {
      // this block also sums the tile-kernel energy partials k = blockIdx.x (mod gridDim.x)
      for (int k = blockIdx.x + threadIdx.x * gridDim.x; k < nep; k += blockDim.x * gridDim.x) vals[0] += epart[k];
    }
    double t[NV], r[NV];
    block_sum_n<NV>(vals, sh, t);
    if (grid_reduce<NV>(t, npart, ctr, sh, r) && threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) red[k] = r[k];
      if (phi2) *phi2 = r[0];
    }
  } else {
    double bs = block_sum(dotv, sh), tot;
    if (grid_reduce<1>(&bs, npart, ctr, sh, &tot) && threadIdx.x == 0) cg_set_alpha(cg, tot);
  }
}

template <int D, typename R>
__global__ void __launch_bounds__(64 * kMergeTiles) k_merge_heat(Dev<R> d, TileLists tl, int ntiles,
                                                                 const R* tpart, const R* T, R* out, const int* done,
                                                                 double* npart, unsigned* ctr, CgScal* cg,
                                                                 PUpd<R> pu) {
  constexpr int RN = TileGeo<D>::RN;
  __shared__ double sh[kRedSh];
  if (done && *done) return;
  const int ti = xcd_slot(blockIdx.x, kMergeRun) * kMergeTiles + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double dotv = 0;
  if (ti < ntiles) {
    const int tile = d.tile_list[ti];
    const int node = tile * kTileNodes + lane;
    MergeSrc<D> ms;
    merge_sources_tab<D>(ti, lane, tl.nbr, ms);
    R acc = 0;
    R val[1 << D];
#pragma unroll
    for (int j = 0; j < (1 << D); ++j)
      val[j] = ms.slot[j] >= 0 ? tpart[(size_t)ms.slot[j] * RN + ms.rn[j]] : R(0);
#pragma unroll
    for (int j = 0; j < (1 << D); ++j) acc += val[j];
    bool dof = d.gfree[node] & 0x80;
    R Ti = T[node];
    const R mn = d.gm[node];   // loaded before the store below, which may alias it for the compiler
    if (pu.z) {
      Ti = cg_dir(pu.z[node], pu.beta(), Ti);
      pu.p[node] = Ti;
    }
    R o = dof ? d.cp / d.dt * mn * Ti + acc : R(0);
    out[node] = o;
    if (dof) dotv = (double)Ti * (double)o;
  }
  if (!cg) return;
  double bs = block_sum(dotv, sh), tot;
  if (grid_reduce<1>(&bs, npart, ctr, sh, &tot) && threadIdx.x == 0) cg_set_alpha(cg, tot);
}

// P2G merge and grid set-up (degrees of freedom, v^n, T^n, constraints, diagonals, heat
// right side).
template <int D, typename R>
__global__ void __launch_bounds__(64) k_merge_p2g(Dev<R> d, TileLists tl, const R* tpart, int* nbr_out) {
  constexpr int RN = TileGeo<D>::RN;
  using FI = P2GF<D>;
  constexpr int NF = FI::NF;
  const int tile = d.tile_list[blockIdx.x];
  const int lane = threadIdx.x;
  const int node = tile * kTileNodes + lane;
  const int nn = d.nn;
  int i[3] = {0, 0, 0};
  tiled_coords<D>(tile, lane, d.nt, i);
  MergeSrc<D> ms;
  merge_sources<D>(tile, lane, d.nt, tl.ctile_slot, ms);
  // this node tile's row of the neighbour-slot table, for the later merges of the step
  if (lane < (D == 3 ? 27 : 9)) {
    const int o[3] = {lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1};
    int T[3] = {0, 0, 0};
    tiled_coords<D>(tile, 0, d.nt, T);
    bool in = true;
    int ct = 0, mul = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int C = T[a] / TileGeo<D>::E + o[a];
      in = in && C >= 0 && C < d.nt;
      ct += mul * C;
      mul *= d.nt;
    }
    nbr_out[(size_t)blockIdx.x * kNbr + lane] = in ? tl.ctile_slot[ct] : -1;
  }
  R v[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) v[f] = 0;
#pragma unroll
  for (int j = 0; j < (1 << D); ++j) {
    if (ms.slot[j] < 0) continue;
    R t[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) t[f] = tpart[((size_t)ms.slot[j] * RN + ms.rn[j]) * NF + f];
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] += t[f];
  }
  const R m = v[FI::M], W = v[FI::W], WT = v[FI::WT], E = v[FI::E], ET = v[FI::ET];
  const bool dof = m > R(0);
  d.gm[node] = m; d.gW[node] = W; d.gWT[node] = WT; d.gE[node] = E; d.gET[node] = ET;
  R Tn = W > R(0) ? WT / W : (E > R(0) ? ET / E : R(0));
  d.gTn[node] = dof ? Tn : R(0);
  uint8_t fr = dof ? 0x80 : 0;
  R xi[3];
#pragma unroll
  for (int a = 0; a < D; ++a) xi[a] = (R(i[a]) + R(0.5)) * d.dx;
  bool in_slab = d.slab != 0;
#pragma unroll
  for (int a = 0; a < D; ++a) in_slab = in_slab && xi[a] >= d.slab_lo[a] && xi[a] < d.slab_hi[a];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    bool wall = d.wall > 0 && (i[a] < d.wall || i[a] >= d.n - d.wall);
    bool fixed = wall || (in_slab && a == d.slab_axis);
    bool fa = dof && !fixed;
    if (fa) fr |= (uint8_t)(1u << a);
    R mv = v[FI::MV + a];
    d.gmv[a * nn + node] = mv;
    d.gvn[a * nn + node] = dof ? mv / m : R(0);
    d.gdiag[a * nn + node] = fa ? m + v[FI::DG + a] : R(1);
  }
  d.gfree[node] = fr;
  R cm = d.cp / d.dt * m;
  d.hdiag[node] = dof ? cm + v[FI::HD] : R(1);
  d.hrhs[node] = dof ? cm * Tn + v[FI::HR] : R(0);
}

// Active cell tiles (tiles holding any point), in two classes: flag[t] marks the tiles
// with surface samples, flag[ntile + t] the others.  One scan of the 2 ntile flags then
// numbers the tiles with samples first.  Workgroups of the tile kernels start in slot
// order, and the tiles with samples are the costly ones (their samples take the surface
// terms), so this order leaves the cheap tiles to fill the end of a launch.
template <int D, typename R>
__global__ void k_flag_ctiles(Dev<R> d, int* flag, int ntile) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntile) return;
  int cb = t * 64;
  int cnt = d.p_start[cb + 64] - d.p_start[cb];
  int ns = 0;
  if (d.ns) {
    ns = d.s_start[cb + 64] - d.s_start[cb];
    cnt += ns + (d.b_start[cb + 64] - d.b_start[cb]);
  }
  flag[t] = cnt > 0 && ns > 0;
  flag[ntile + t] = cnt > 0 && ns == 0;
}

// Slots of the active tiles from the scan of k_flag_ctiles' flags (pos over 2 ntile + 1).
template <typename R>
__global__ void k_ctile_slots(Dev<R> d, const int* flag, const int* pos, int ntile, int* list, int* slot, int* rng) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntile) return;
  const bool first = flag[t];
  if (first || flag[ntile + t]) {
    int s = first ? pos[t] : pos[ntile + t], cb = t * 64;
    list[s] = t;
    slot[t] = s;
    int* r = rng + 6 * s;
    r[0] = d.p_start[cb]; r[1] = d.p_start[cb + 64];
    r[2] = d.ns ? d.s_start[cb] : 0; r[3] = d.ns ? d.s_start[cb + 64] : 0;
    r[4] = d.ns ? d.b_start[cb] : 0; r[5] = d.ns ? d.b_start[cb + 64] : 0;
  } else {
    slot[t] = -1;
  }
}

}  // namespace mpm
