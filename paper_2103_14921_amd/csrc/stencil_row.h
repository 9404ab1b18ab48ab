// Row coefficients of the 27-point PML operator, shared by the stencil, the
// Galerkin coarse-operator build and the local-operator assembly.
#pragma once
#include "common.h"

// Weights of the edge (i, j), j the neighbour of node i of class cls (1 face,
// 2 edge, 3 corner; j < 0 for a ghost neighbour outside the grid).  With
// per-node weights (adaptive coefficients) the edge's stiffness weight is the
// mean of its two end nodes' (the node's own toward a ghost) and its mass
// coupling the mean of wm_cls sigma at its two ends, so that A = A^T.
static __device__ __forceinline__ double edge_alpha(const OpDev& op, long long i, long long j, int cls) {
  if (!op.wnode) return op.alpha[cls - 1];
  const double ai = op.wnode[i * 8 + cls - 1];
  return j < 0 ? ai : 0.5 * (ai + op.wnode[j * 8 + cls - 1]);
}
static __device__ __forceinline__ z64 edge_mass(const OpDev& op, long long i, long long j, int cls, z64 si, z64 sj) {
  if (!op.wnode) return (0.5 * op.wm[cls]) * (si + sj);
  return 0.5 * (op.wnode[i * 8 + 3 + cls] * si + op.wnode[j * 8 + 3 + cls] * sj);
}
static __device__ __forceinline__ double diag_mass(const OpDev& op, long long i) {
  return op.wnode ? op.wnode[i * 8 + 3] : op.wm[0];
}

// Stiffness part (alpha/h^2) a_e(m) of the edge (i, i+o) with weight alpha.
static __device__ __forceinline__ z64 stiff_coef(const OpDev& op, double alpha, int ix, int iy, int iz, int ox, int oy,
                                                 int oz) {
  const int cls = abs(ox) + abs(oy) + abs(oz);
  const double we = cls == 1 ? 1.0 : (cls == 2 ? 0.5 : 1.0 / 3.0);
  z64 s = mk(1.0, 0.0), inv = mk(0.0, 0.0);
  const int pos[3] = {ix, iy, iz};
  const int od[3] = {ox, oy, oz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (od[d] == 0) {
      s = s * op.xi_int[op.off_int[d] + pos[d]];
    } else {
      const int t = pos[d] + (od[d] > 0 ? 1 : 0);
      s = s * op.xi_half[op.off_half[d] + t];
      inv += we * op.i2_half[op.off_half[d] + t];
    }
  }
  return (alpha * op.h2inv) * (s * inv);
}

// Diagonal of row i: wm1 sigma_i minus the stiffness of its 26 edges, summed in
// offset order (the same terms and order as fine_row's c[13]).
static __device__ __forceinline__ z64 row_diag(const OpDev& op, int ix, int iy, int iz) {
  const long long i = ix + (long long)op.nx * (iy + (long long)op.ny * iz);
  z64 diag = diag_mass(op, i) * op.sigma[i];
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    if (o == 13) continue;
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const int cls = abs(ox) + abs(oy) + abs(oz);
    const int jx = ix + ox, jy = iy + oy, jz = iz + oz;
    const bool inside = jx >= 0 && jx < op.nx && jy >= 0 && jy < op.ny && jz >= 0 && jz < op.nz;
    const long long j = inside ? jx + (long long)op.nx * (jy + (long long)op.ny * jz) : -1;
    diag -= stiff_coef(op, edge_alpha(op, i, j, cls), ix, iy, iz, ox, oy, oz);
  }
  return diag;
}

// Coefficients of row i = (ix, iy, iz) for the products into c[0..26], by L
// lanes per node: lane q computes the offsets q, q + L, ... (zero towards a
// neighbour outside the grid; all zero when !valid) and lane 0 also the
// stored diagonal.  Each coefficient is computed on its own, so every lane
// count gives the same values and every product sees the same operator.
template <int L>
static __device__ __forceinline__ void row_coefs(const OpDev& op, bool valid, int ix, int iy, int iz, int q, z64* c) {
  if (!valid) {
    for (int o = q; o < 27; o += L) c[o] = mk(0.0, 0.0);
    return;
  }
  const long long i = ix + (long long)op.nx * (iy + (long long)op.ny * iz);
  const z64 si = op.sigma[i];
  const bool flat = op.flat[op.off_int[0] + ix] && op.flat[op.off_int[1] + iy] && op.flat[op.off_int[2] + iz];
  for (int o = q; o < 27; o += L) {
    if (o == 13) {
      c[13] = op.diag[i];
      continue;
    }
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const int jx = ix + ox, jy = iy + oy, jz = iz + oz;
    if (jx < 0 || jx >= op.nx || jy < 0 || jy >= op.ny || jz < 0 || jz >= op.nz) {
      c[o] = mk(0.0, 0.0);
      continue;
    }
    const int cls = abs(ox) + abs(oy) + abs(oz);
    const long long j = jx + (long long)op.nx * (jy + (long long)op.ny * jz);
    const double al = edge_alpha(op, i, j, cls);
    const z64 st = flat ? mk(al * op.h2inv, 0.0) : stiff_coef(op, al, ix, iy, iz, ox, oy, oz);
    c[o] = st + edge_mass(op, i, j, cls, si, op.sigma[j]);
  }
}

// Full row i of A: c[o] for the 27 offsets (zero for ghost neighbours), c[13] the diagonal.
static __device__ __forceinline__ void fine_row(const OpDev& op, int ix, int iy, int iz, z64* c) {
  const long long i = ix + (long long)op.nx * (iy + (long long)op.ny * iz);
  const z64 si = op.sigma[i];
  z64 diag = diag_mass(op, i) * si;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    if (o == 13) continue;
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const int cls = abs(ox) + abs(oy) + abs(oz);
    const int jx = ix + ox, jy = iy + oy, jz = iz + oz;
    const bool inside = jx >= 0 && jx < op.nx && jy >= 0 && jy < op.ny && jz >= 0 && jz < op.nz;
    const long long j = inside ? jx + (long long)op.nx * (jy + (long long)op.ny * jz) : -1;
    const z64 st = stiff_coef(op, edge_alpha(op, i, j, cls), ix, iy, iz, ox, oy, oz);
    diag -= st;
    c[o] = inside ? st + edge_mass(op, i, j, cls, si, op.sigma[j]) : mk(0.0, 0.0);
  }
  c[13] = diag;
}

