// Row coefficients of the 27-point PML operator, shared by the stencil, the
// Galerkin coarse-operator build and the local-operator assembly.
#pragma once
#include "common.h"

// Coefficient of the edge (i, i+o) without the mass term, and the mass weight.
// Returns the stiffness part (alpha/h^2) a_e(m).
static __device__ __forceinline__ z64 stiff_coef(const OpDev& op, int ix, int iy, int iz, int ox, int oy, int oz) {
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
  return (op.alpha[cls - 1] * op.h2inv) * (s * inv);
}

// Full row i of A: c[o] for the 27 offsets (zero for ghost neighbours), c[13] the diagonal.
static __device__ __forceinline__ void fine_row(const OpDev& op, int ix, int iy, int iz, z64* c) {
  const long long i = ix + (long long)op.nx * (iy + (long long)op.ny * iz);
  const z64 si = op.sigma[i];
  z64 diag = op.wm[0] * si;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    if (o == 13) continue;
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const int cls = abs(ox) + abs(oy) + abs(oz);
    const z64 st = stiff_coef(op, ix, iy, iz, ox, oy, oz);
    diag -= st;
    const int jx = ix + ox, jy = iy + oy, jz = iz + oz;
    if (jx >= 0 && jx < op.nx && jy >= 0 && jy < op.ny && jz >= 0 && jz < op.nz) {
      const z64 sj = op.sigma[jx + (long long)op.nx * (jy + (long long)op.ny * jz)];
      c[o] = st + (0.5 * op.wm[cls]) * (si + sj);
    } else {
      c[o] = mk(0.0, 0.0);
    }
  }
  c[13] = diag;
}

