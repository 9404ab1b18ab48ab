// Medium preparation, the matrix-free 27-point PML stencil, the Galerkin
// coarse operator E = Z^T A Z and the coarse transfers.
//
// Operator (eq. eqh / eq. eq1; symmetric stretched-coordinate form): for each
// of the 26 neighbours j = i + o of node i, with e = o, cls = |ox|+|oy|+|oz|,
//   A[i, j] = (alpha_cls/h^2) a_e(m) + wm_cls (sigma_i + sigma_j)/2,
//   a_e(m)  = s(m) * sum_{d: o_d != 0} (1/cls) / xi_d(m_d)^2,   s = xi_x xi_y xi_z,
// m the midpoint of the edge i-j, and
//   A[i, i] = -sum_o (alpha_cls/h^2) a_e(m) + wm1 sigma_i,   sigma = s k^2,
// ghost neighbours outside the grid contributing to the diagonal only.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>
#include "kernels.h"
#include "stencil_row.h"

namespace {

__global__ void k_vmax(const z64* __restrict__ c, long long n, double* out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, c[i].re);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

struct AxisTables {
  AxisPml ax[3];
  int off_int[3], off_half[3];
};

__device__ double pml_gamma(const AxisPml& a, double t, double h, double vmax, double R) {
  // gamma(t) = gmax (dist/L)^2, gmax = 3 vmax/(2L) ln(1/R), L = npml h; the high side wins on overlap
  double g = 0.0;
  if (a.lo > 0 && t < (double)a.lo) {
    double L = a.lo * h;
    double gmax = 1.5 * vmax / L * log(1.0 / R);
    double d = ((a.lo - t) * h) / L;
    g = gmax * d * d;
  }
  if (a.hi > 0 && t > (double)(a.n - 1 - a.hi)) {
    double L = a.hi * h;
    double gmax = 1.5 * vmax / L * log(1.0 / R);
    double d = ((t - (a.n - 1 - a.hi)) * h) / L;
    g = gmax * d * d;
  }
  return g;
}

__global__ void k_pml_tables(AxisTables tb, double h, double omega, double R, const double* vmax_p,
                             z64* xi_int, z64* xi_half, z64* i2_int, z64* i2_half, uint8_t* flat) {
  const int d = blockIdx.y;
  const AxisPml a = tb.ax[d];
  const double vmax = vmax_p[0];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= a.n) {
    // half position j - 1/2 for j = t
    z64 xh = mk(1.0, pml_gamma(a, t - 0.5, h, vmax, R) / omega);
    xi_half[tb.off_half[d] + t] = xh;
    i2_half[tb.off_half[d] + t] = cinv(xh * xh);
  }
  if (t < a.n) {
    z64 xi = mk(1.0, pml_gamma(a, (double)t, h, vmax, R) / omega);
    xi_int[tb.off_int[d] + t] = xi;
    i2_int[tb.off_int[d] + t] = cinv(xi * xi);
    bool f = pml_gamma(a, t - 0.5, h, vmax, R) == 0.0 && pml_gamma(a, (double)t, h, vmax, R) == 0.0 &&
             pml_gamma(a, t + 0.5, h, vmax, R) == 0.0;
    flat[tb.off_int[d] + t] = f ? 1 : 0;
  }
}

__global__ void k_sigma(OpDev op, const z64* __restrict__ c, double omega, z64* sigma) {
  const long long n = (long long)op.nx * op.ny * op.nz;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    int ix = (int)(i % op.nx);
    long long q = i / op.nx;
    int iy = (int)(q % op.ny);
    int iz = (int)(q / op.ny);
    z64 s = op.xi_int[op.off_int[2] + iz] * op.xi_int[op.off_int[1] + iy] * op.xi_int[op.off_int[0] + ix];
    z64 k = cdiv(mk(omega, 0.0), c[i]);
    sigma[i] = s * (k * k);
  }
}

// Adaptive coefficients: per node G = Re(c)/(f h) points per wavelength, the
// weight set interpolated linearly in G between the table entries around it
// (entry j at g0 + j dg, [n][7] = w1 w2 w3 wm1 wm2 wm3 wm4; clamped at the
// ends), stored as alpha_face, alpha_edge, alpha_corner, wm1..wm4.
__global__ void k_node_weights(const z64* __restrict__ c, long long n, double freq, double h, const double* __restrict__ tab,
                               int ntab, double g0, double dg, double* __restrict__ wnode) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double G = c[i].re / (freq * h);
    const double x = fmin(fmax((G - g0) / dg, 0.0), ntab - 1.0);
    const int j = min((int)floor(x), ntab - 2);
    const double t = x - j;
    double w[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) w[q] = (1.0 - t) * tab[j * 7 + q] + t * tab[(j + 1) * 7 + q];
    double* o = wnode + i * 8;
    o[0] = w[0] + w[1] / 3.0;
    o[1] = w[1] / 6.0;
    o[2] = w[2] / 4.0;
    o[3] = w[3];
    o[4] = w[4];
    o[5] = w[5];
    o[6] = w[6];
    o[7] = 0.0;
  }
}

}  // namespace

void launch_node_weights(const z64* c, long long n, double freq, double h, const double* tab, int ntab, double g0,
                         double dg, double* wnode, hipStream_t s) {
  hipLaunchKernelGGL(k_node_weights, dim3((unsigned)std::min<long long>(ceil_div(n, 256), 16384)), dim3(256), 0, s, c, n,
                     freq, h, tab, ntab, g0, dg, wnode);
}

namespace {

// Stencil y = A x (or y = b - A x).  A block of 256 threads owns nb = 256/nrhs
// (at most 64) consecutive nodes: phase 1 computes the 27 row coefficients of each node
// once into LDS (shared by all right-hand sides), phase 2 maps one thread to
// each (node, right-hand side) pair, right-hand side fastest, so that the
// neighbour loads of a wave are contiguous.
__global__ void __launch_bounds__(256) k_stencil2(OpDev op, int nrhs, const z64* __restrict__ x,
                                                  z64* __restrict__ y, const z64* __restrict__ b) {
  extern __shared__ z64 lds_coef[];
  const long long n = (long long)op.nx * op.ny * op.nz;
  const int nb = nrhs >= 256 ? 1 : (nrhs >= 4 ? 256 / nrhs : 64);
  z64(*coef)[27] = reinterpret_cast<z64(*)[27]>(lds_coef);
  const long long i0 = (long long)blockIdx.x * nb;
  const int tid = threadIdx.x;
  // phase 1: coefficients (node a, offset o)
  for (int t = tid; t < nb * 4; t += 256) {  // four lanes per node
    const int a = t >> 2;
    const long long i = i0 + a;
    const long long ic = i < n ? i : 0;
    row_coefs<4>(op, i < n, (int)(ic % op.nx), (int)((ic / op.nx) % op.ny), (int)(ic / op.nx / op.ny), t & 3, coef[a]);
  }
  __syncthreads();
  // phase 2: one thread per (node, rhs)
  for (int t = tid; t < nb * nrhs; t += 256) {
    const int a = t / nrhs, r = t % nrhs;
    const long long i = i0 + a;
    if (i >= n) continue;
    const int ix = (int)(i % op.nx);
    const long long q = i / op.nx;
    const int iy = (int)(q % op.ny);
    const int iz = (int)(q / op.ny);
    // ghost neighbours have zero coefficients: their loads are clamped into the
    // grid and issued with the others (no branches, all 27 loads in flight)
    z64 acc = mk(0.0, 0.0);
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      const int jx = min(max(ix + o % 3 - 1, 0), op.nx - 1);
      const int jy = min(max(iy + (o / 3) % 3 - 1, 0), op.ny - 1);
      const int jz = min(max(iz + o / 9 - 1, 0), op.nz - 1);
      const long long j = jx + (long long)op.nx * (jy + (long long)op.ny * jz);
      cfma(acc, coef[a][o], x[j * nrhs + r]);
    }
    if (b) y[i * nrhs + r] = b[i * nrhs + r] - acc;
    else y[i * nrhs + r] = acc;
  }
}

// Row-tiled 27-point products (batches of 8 or more right-hand sides).  A
// block owns a segment of at most TW consecutive nodes of one grid row (iy, iz)
// and all right-hand sides.  Phase 1 puts the 27 coefficients of each node in
// LDS (zero towards neighbours outside the grid); phase 2 gives each thread NXT
// consecutive nodes of one right-hand side: for each of the nine neighbour
// rows it loads NXT + 2 values once and uses them for all NXT outputs, where a
// node-per-thread product issues 27 vector loads per output.  NXT (2, 4 or 8)
// is chosen per grid and batch by the autotuner below; every choice sums the
// 27 taps of an output in the same order, so results do not depend on it.
constexpr int TW = 64;

struct RowTile {
  int iy, iz, x0, w;
};
// Tile order: bands of ROW_BAND grid rows (y), each swept through all planes
// (z), segments of a row fastest.  The workgroups resident on one XCD then
// cover a compact (y, z) patch, whose nine neighbour rows per tile largely
// overlap in that XCD's L2 (plane-by-plane order re-fetches each input row
// about four times from beyond L2; this order about one and a half).
constexpr int ROW_BAND = 8;
template <int NXT>
__device__ __forceinline__ RowTile row_tile(int nx, int ny, int nz) {
  const int nt = (nx + TW - 1) / TW;
  const int tw = ((nx + nt - 1) / nt + NXT - 1) / NXT * NXT;  // balanced segment width, multiple of NXT
  const long long lb = xcd_contiguous(blockIdx.x, gridDim.x);
  const long long per_band = (long long)ROW_BAND * nz * nt;
  const int band = (int)(lb / per_band);
  long long rem = lb - band * per_band;
  const int tx = (int)(rem % nt);
  rem /= nt;
  const int nyb = min(ROW_BAND, ny - band * ROW_BAND);  // the last band may be narrower
  RowTile t;
  t.iy = band * ROW_BAND + (int)(rem % nyb);
  t.iz = (int)(rem / nyb);
  t.x0 = tx * tw;
  t.w = min(tw, nx - t.x0);
  return t;
}

// y = cf x (or b - cf x) on the tile; cf[a][o] holds node x0 + a's row.
template <int NXT>
__device__ __forceinline__ void tile_product(const RowTile& t, int nx, int ny, int nz, int nrhs,
                                             const z64 (*cf)[27], const z64* __restrict__ x, z64* __restrict__ y,
                                             const z64* __restrict__ b) {
  const int ngr = (t.w + NXT - 1) / NXT;
  for (int item = threadIdx.x; item < ngr * nrhs; item += blockDim.x) {
    const int g = item / nrhs, r = item % nrhs;
    const int xa = t.x0 + g * NXT;
    z64 acc[NXT];
#pragma unroll
    for (int m = 0; m < NXT; ++m) acc[m] = mk(0.0, 0.0);
    // the nine neighbour rows (dz, dy) in order; latency is hidden by the
    // other waves of the compute unit
#pragma unroll 1
    for (int k = 0; k < 9; ++k) {
      const int jz = min(max(t.iz + k / 3 - 1, 0), nz - 1), jy = min(max(t.iy + k % 3 - 1, 0), ny - 1);
      const z64* xr = x + (long long)nx * (jy + (long long)ny * jz) * nrhs + r;
      z64 v[NXT + 2];
#pragma unroll
      for (int q = 0; q < NXT + 2; ++q) v[q] = xr[(long long)min(max(xa - 1 + q, 0), nx - 1) * nrhs];
      const int ob = 3 * k;
#pragma unroll
      for (int m = 0; m < NXT; ++m)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) cfma(acc[m], cf[g * NXT + m][ob + dx], v[m + dx]);
    }
    const long long rowi = (long long)nx * (t.iy + (long long)ny * t.iz);
#pragma unroll
    for (int m = 0; m < NXT; ++m) {
      if (xa + m >= t.x0 + t.w) break;
      const long long e = (rowi + xa + m) * nrhs + r;
      y[e] = b ? b[e] - acc[m] : acc[m];
    }
  }
}

template <int NXT>
__global__ void __launch_bounds__(256) k_stencil_rows(OpDev op, int nrhs, const z64* __restrict__ x,
                                                      z64* __restrict__ y, const z64* __restrict__ b) {
  __shared__ z64 cf[TW][27];
  const RowTile t = row_tile<NXT>(op.nx, op.ny, op.nz);
  // phase 1: the tile's row coefficients, four lanes per node
  const int a = threadIdx.x >> 2;
  row_coefs<4>(op, a < t.w, t.x0 + a, t.iy, t.iz, threadIdx.x & 3, cf[a]);
  __syncthreads();
  tile_product<NXT>(t, op.nx, op.ny, op.nz, nrhs, cf, x, y, b);
}

template <int NXT>
__global__ void __launch_bounds__(256) k_coarse_spmv_rows(int ncx, int ncy, int ncz, const z64* __restrict__ E,
                                                          int nrhs, const z64* __restrict__ x, z64* __restrict__ y) {
  __shared__ z64 cf[TW][27];
  const RowTile t = row_tile<NXT>(ncx, ncy, ncz);
  const long long rowi = (long long)ncx * (t.iy + (long long)ncy * t.iz);
  for (int e = threadIdx.x; e < TW * 27; e += blockDim.x) {
    const int a = e / 27, o = e % 27;
    z64 c = mk(0.0, 0.0);
    if (a < t.w) {
      const int jx = t.x0 + a + o % 3 - 1, jy = t.iy + (o / 3) % 3 - 1, jz = t.iz + o / 9 - 1;
      if (jx >= 0 && jx < ncx && jy >= 0 && jy < ncy && jz >= 0 && jz < ncz) c = E[(rowi + t.x0 + a) * 27 + o];
    }
    cf[a][o] = c;
  }
  __syncthreads();
  tile_product<NXT>(t, ncx, ncy, ncz, nrhs, cf, x, y, nullptr);
}

// Plane-marching 27-point products for batches of 16 k right-hand sides.  A
// workgroup owns a segment of MW = (256 / RW) NXT consecutive nodes of one grid
// row and MZ planes of it, for RW right-hand sides (one block of the batch):
// thread (g, r) keeps NXT consecutive nodes of right-hand side r and marches
// through the planes, loading each plane's three neighbour rows once (NXT + 2
// values each) and adding their terms to the outputs of the planes below, at
// and above it, whose accumulators rotate; the output of plane p - 1 is
// complete once plane p is in.  A row-tiled product loads nine neighbour rows
// per output plane, this form three.  The row coefficients of the three planes
// in flight sit in an LDS ring: generated (row_coefs, as the row-tiled product
// does, eight lanes per node) or, for E, copied from its stored rows.  Every
// output sums its 27 terms in offset order, as the row-tiled product, so the
// results are bitwise identical (terms with a neighbour plane outside the grid
// have zero coefficients and are skipped).
constexpr int MZ = 16;
template <int NXT, int RW>
struct March {
  static constexpr int MW = (256 / RW) * NXT;  // nodes per segment
};
struct MarchTile {
  int x0, w, iy, z0, z1;
};
template <int NXT, int RW>
__device__ __forceinline__ MarchTile march_tile(int nx, int ny, int nz) {
  constexpr int MW = March<NXT, RW>::MW;
  const int nt = (nx + MW - 1) / MW;
  // segments of a row fastest, then rows, then plane chunks; XCDs take contiguous ranges
  const long long lb = xcd_contiguous(blockIdx.x, gridDim.x);
  MarchTile t;
  const int tx = (int)(lb % nt);
  t.iy = (int)((lb / nt) % ny);
  t.z0 = (int)(lb / ((long long)nt * ny)) * MZ;
  t.z1 = min(t.z0 + MZ, nz);
  t.x0 = tx * MW;
  t.w = min(MW, nx - t.x0);
  return t;
}
template <int NXT, int RW>
static unsigned march_tiles(int nx, int ny, int nz) {
  constexpr int MW = March<NXT, RW>::MW;
  return (unsigned)((long long)((nx + MW - 1) / MW) * ny * ((nz + MZ - 1) / MZ));
}

// E == nullptr: the fine operator's rows, generated; else E's stored rows [node][27]
template <int NXT, int RW>
__global__ void __launch_bounds__(256) k_march(OpDev op, int nx, int ny, int nz, const z64* __restrict__ E, int nrhs,
                                               const z64* __restrict__ x, z64* __restrict__ y,
                                               const z64* __restrict__ b) {
  constexpr int MW = March<NXT, RW>::MW;
  __shared__ z64 ring[3][MW][27];
  const MarchTile t = march_tile<NXT, RW>(nx, ny, nz);
  const int g = threadIdx.x / RW, r = (int)blockIdx.y * RW + threadIdx.x % RW;
  const int xa = t.x0 + g * NXT;
  const long long plane = (long long)nx * ny;
  z64 acc[3][NXT];  // outputs of planes p - 1, p, p + 1
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int m = 0; m < NXT; ++m) acc[a][m] = mk(0.0, 0.0);
  for (int p = t.z0 - 1; p <= t.z1; ++p) {
    __syncthreads();  // the slot refilled below was last read in the previous step
    const int zn = p + 1;
    if (zn >= t.z0 && zn < t.z1) {
      z64(*slot)[27] = ring[zn % 3];
      if (E == nullptr) {
        constexpr int L = 256 / MW >= 8 ? 8 : 4;  // lanes per node
        const int a = threadIdx.x / L;
        if (a < MW) row_coefs<L>(op, a < t.w, t.x0 + a, t.iy, zn, threadIdx.x % L, slot[a]);
      } else {
        const long long rowi = (long long)nx * (t.iy + (long long)ny * zn);
        for (int e = threadIdx.x; e < MW * 27; e += 256) {
          const int a = e / 27, o = e % 27;
          z64 c = mk(0.0, 0.0);
          if (a < t.w) {
            const int jx = t.x0 + a + o % 3 - 1, jy = t.iy + (o / 3) % 3 - 1, jz = zn + o / 9 - 1;
            if (jx >= 0 && jx < nx && jy >= 0 && jy < ny && jz >= 0 && jz < nz) c = E[(rowi + t.x0 + a) * 27 + o];
          }
          slot[a][o] = c;
        }
      }
    }
    __syncthreads();
    if (p >= 0 && p < nz && g * NXT < t.w) {
      z64 v[3][NXT + 2];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int jy = min(max(t.iy + k - 1, 0), ny - 1);
        const z64* xr = x + (p * plane + (long long)jy * nx) * nrhs + r;
#pragma unroll
        for (int q = 0; q < NXT + 2; ++q) v[k][q] = xr[(long long)min(max(xa - 1 + q, 0), nx - 1) * nrhs];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int zt = p - 1 + a;  // output plane; this plane is its neighbour at dz = 1 - a
        if (zt < t.z0 || zt >= t.z1) continue;
        const z64(*cf)[27] = ring[zt % 3];
        const int ob = 9 * (2 - a);
#pragma unroll
        for (int m = 0; m < NXT; ++m)
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) cfma(acc[a][m], cf[g * NXT + m][ob + 3 * k + dx], v[k][m + dx]);
      }
    }
    const int zo = p - 1;
    if (zo >= t.z0 && zo < t.z1) {
      const long long rowi = zo * plane + (long long)t.iy * nx;
#pragma unroll
      for (int m = 0; m < NXT; ++m) {
        if (xa + m >= t.x0 + t.w) break;
        const long long e = (rowi + xa + m) * nrhs + r;
        y[e] = b ? b[e] - acc[0][m] : acc[0][m];
      }
    }
#pragma unroll
    for (int m = 0; m < NXT; ++m) {
      acc[0][m] = acc[1][m];
      acc[1][m] = acc[2][m];
      acc[2][m] = mk(0.0, 0.0);
    }
  }
}

// E[I][o] = sum_i sum_j Z[i,I] A[i,j] Z[j,I+o]; one thread per coarse node I,
// its 27 sums in LDS (indexed at run time), the fine row in registers.
constexpr int BUILD_E_BLOCK = 64;
__global__ void __launch_bounds__(BUILD_E_BLOCK) k_build_E(OpDev op, int ncx, int ncy, int ncz, z64* __restrict__ E) {
  __shared__ z64 acc_s[BUILD_E_BLOCK][27];
  const long long nc = (long long)ncx * ncy * ncz;
  const long long I = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int cx = (int)(I % ncx);
  const int cy = (int)((I / ncx) % ncy);
  const int cz = (int)(I / ((long long)ncx * ncy));
  z64* acc = acc_s[threadIdx.x];
  for (int o = 0; o < 27; ++o) acc[o] = mk(0.0, 0.0);
  z64 row[27];
  for (int dz = -1; dz <= 1; ++dz) {
    const int iz = 2 * cz + dz;
    if (iz < 0 || iz >= op.nz) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int iy = 2 * cy + dy;
      if (iy < 0 || iy >= op.ny) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int ix = 2 * cx + dx;
        if (ix < 0 || ix >= op.nx) continue;
        const double wi = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0);
        fine_row(op, ix, iy, iz, row);
#pragma unroll
        for (int o = 0; o < 27; ++o) {
          const int jx = ix + o % 3 - 1, jy = iy + (o / 3) % 3 - 1, jz = iz + o / 9 - 1;
          if (jx < 0 || jx >= op.nx || jy < 0 || jy >= op.ny || jz < 0 || jz >= op.nz) continue;
          const z64 a = wi * row[o];
          // coarse nodes J with Z[j, J] != 0 along each axis
          int jxs[2], jys[2], jzs[2], nxs, nys, nzs;
          double wxs[2], wys[2], wzs[2];
          if ((jx & 1) == 0) { jxs[0] = jx / 2; wxs[0] = 1.0; nxs = 1; }
          else { jxs[0] = (jx - 1) / 2; jxs[1] = (jx + 1) / 2; wxs[0] = wxs[1] = 0.5; nxs = 2; }
          if ((jy & 1) == 0) { jys[0] = jy / 2; wys[0] = 1.0; nys = 1; }
          else { jys[0] = (jy - 1) / 2; jys[1] = (jy + 1) / 2; wys[0] = wys[1] = 0.5; nys = 2; }
          if ((jz & 1) == 0) { jzs[0] = jz / 2; wzs[0] = 1.0; nzs = 1; }
          else { jzs[0] = (jz - 1) / 2; jzs[1] = (jz + 1) / 2; wzs[0] = wzs[1] = 0.5; nzs = 2; }
          for (int az = 0; az < nzs; ++az) {
            if (jzs[az] >= ncz) continue;
            for (int ay = 0; ay < nys; ++ay) {
              if (jys[ay] >= ncy) continue;
              for (int ax = 0; ax < nxs; ++ax) {
                if (jxs[ax] >= ncx) continue;
                const int oo = (jzs[az] - cz + 1) * 9 + (jys[ay] - cy + 1) * 3 + (jxs[ax] - cx + 1);
                acc[oo] += (wxs[ax] * wys[ay] * wzs[az]) * a;
              }
            }
          }
        }
      }
    }
  }
  for (int o = 0; o < 27; ++o) E[I * 27 + o] = acc[o];
}

// y = E x on the coarse grid: one thread per (coarse node, rhs), rhs fastest;
// the 27 stored coefficients of a node are shared (broadcast) by its rhs lanes.
__global__ void __launch_bounds__(256) k_coarse_spmv2(int ncx, int ncy, int ncz, const z64* __restrict__ E, int nrhs,
                                                      const z64* __restrict__ x, z64* __restrict__ y) {
  const long long nc = (long long)ncx * ncy * ncz;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= nc * nrhs) return;
  const long long I = t / nrhs;
  const int r = (int)(t % nrhs);
  const int cx = (int)(I % ncx);
  const int cy = (int)((I / ncx) % ncy);
  const int cz = (int)(I / ((long long)ncx * ncy));
  const z64* e = E + I * 27;
  z64 acc = mk(0.0, 0.0);
  // branch-free: indices clamped into the grid, taps leaving it masked
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int ux = cx + o % 3 - 1, uy = cy + (o / 3) % 3 - 1, uz = cz + o / 9 - 1;
    const bool in = ux >= 0 && ux < ncx && uy >= 0 && uy < ncy && uz >= 0 && uz < ncz;
    const int jx = min(max(ux, 0), ncx - 1), jy = min(max(uy, 0), ncy - 1), jz = min(max(uz, 0), ncz - 1);
    const long long J = jx + (long long)ncx * (jy + (long long)ncy * jz);
    const z64 c = e[o];
    cfma(acc, in ? c : mk(0.0, 0.0), x[J * nrhs + r]);
  }
  y[t] = acc;
}

// c[I] = sum_i Z[i, I] r[i]   (Z^T, full weighting with weights 1, 1/2 per axis)
// Grid (ceil(ncx nrhs / 256), ncy, ncz): a thread per (coarse node, column) of one coarse grid row.
__global__ void k_restrict(int nx, int ny, int nz, int nrhs, const z64* __restrict__ rf, z64* __restrict__ c) {
  const int ncx = (nx + 1) / 2, ncy = (ny + 1) / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncx * nrhs) return;
  const int cx = t / nrhs, r = t % nrhs, cy = blockIdx.y, cz = blockIdx.z;
  const long long I = cx + (long long)ncx * (cy + (long long)ncy * cz);
  z64 acc = mk(0.0, 0.0);
  // branch-free: fine indices clamped into the grid, weights of taps leaving it zero
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    const int uz = 2 * cz + dz, iz = min(max(uz, 0), nz - 1);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int uy = 2 * cy + dy, iy = min(max(uy, 0), ny - 1);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int ux = 2 * cx + dx, ix = min(max(ux, 0), nx - 1);
        const bool in = ux >= 0 && ux < nx && uy >= 0 && uy < ny && uz >= 0 && uz < nz;
        const double w = in ? (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0) : 0.0;
        acc += w * rf[(ix + (long long)nx * (iy + (long long)ny * iz)) * nrhs + r];
      }
    }
  }
  c[I * nrhs + r] = acc;
}

// q[i] = sum_I Z[i, I] c[I]   (trilinear prolongation)
// Grid (ceil(nx nrhs / 256), ny, nz): a thread per (fine node, column) of one fine grid row.
__global__ void k_prolong(int nx, int ny, int nz, int nrhs, const z64* __restrict__ c, z64* __restrict__ q) {
  const int ncx = (nx + 1) / 2, ncy = (ny + 1) / 2, ncz = (nz + 1) / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nx * nrhs) return;
  const int ix = t / nrhs, r = t % nrhs, iy = blockIdx.y, iz = blockIdx.z;
  const long long i = ix + (long long)nx * (iy + (long long)ny * iz);
  // two coarse taps per axis: (i - 1)/2 and (i + 1)/2 with weight 1/2 each for
  // odd i; i/2 with weight 1 (and a zero-weight second tap) for even i; taps
  // beyond the coarse grid get weight zero and a clamped index
  int xs[2], ys[2], zs[2];
  double wx[2], wy[2], wz[2];
  auto taps = [](int i, int nc, int* js, double* ws) {
    const bool odd = i & 1;
    js[0] = i >> 1;
    ws[0] = odd ? 0.5 : 1.0;
    const int j1 = (i + 1) >> 1;
    js[1] = min(j1, nc - 1);
    ws[1] = (odd && j1 < nc) ? 0.5 : 0.0;
  };
  taps(ix, ncx, xs, wx);
  taps(iy, ncy, ys, wy);
  taps(iz, ncz, zs, wz);
  z64 acc = mk(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
      for (int cc = 0; cc < 2; ++cc)
        acc += (wz[a] * wy[b2] * wx[cc]) * c[(xs[cc] + (long long)ncx * (ys[b2] + (long long)ncy * zs[a])) * nrhs + r];
  q[i * nrhs + r] = acc;
}

// Row diagonals A[i, i] (set-up), one thread per node.
__global__ void __launch_bounds__(256) k_row_diag(OpDev op, z64* __restrict__ diag) {
  const long long n = (long long)op.nx * op.ny * op.nz;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
    const int ix = (int)(i % op.nx), iy = (int)((i / op.nx) % op.ny), iz = (int)(i / op.nx / op.ny);
    diag[i] = row_diag(op, ix, iy, iz);
  }
}

}  // namespace

void launch_row_diag(const OpDev& op, z64* diag, hipStream_t s) {
  const long long n = (long long)op.nx * op.ny * op.nz;
  hipLaunchKernelGGL(k_row_diag, dim3((unsigned)std::min<long long>(ceil_div(n, 256), 65536)), dim3(256), 0, s, op,
                     diag);
}

void launch_vmax(const z64* c, long long n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_vmax, dim3(1), dim3(1024), 0, s, c, n, out);
}

void launch_pml_tables(const AxisPml ax[3], double h, double omega, double R, const double* vmax,
                       z64* xi_int, z64* xi_half, z64* i2_int, z64* i2_half, uint8_t* flat,
                       hipStream_t s) {
  AxisTables tb;
  int oi = 0, oh = 0, nmax = 0;
  for (int d = 0; d < 3; ++d) {
    tb.ax[d] = ax[d];
    tb.off_int[d] = oi;
    tb.off_half[d] = oh;
    oi += ax[d].n;
    oh += ax[d].n + 1;
    nmax = ax[d].n + 1 > nmax ? ax[d].n + 1 : nmax;
  }
  hipLaunchKernelGGL(k_pml_tables, dim3((unsigned)ceil_div(nmax, 256), 3), dim3(256), 0, s, tb, h, omega,
                     R, vmax, xi_int, xi_half, i2_int, i2_half, flat);
}

void launch_sigma(const OpDev& op, const z64* c, double omega, hipStream_t s) {
  hipLaunchKernelGGL(k_sigma, dim3(2048), dim3(256), 0, s, op, c, omega, const_cast<z64*>(op.sigma));
}

static unsigned row_tiles(int nx, int ny, int nz) {
  return (unsigned)((long long)((nx + TW - 1) / TW) * ny * nz);
}

// Autotuned nodes per thread of the row-tiled products, per grid and batch:
// every candidate is timed twice on the live input at the first application
// outside a stream capture (the products are idempotent) and the fastest kept.
namespace {
struct RowKey {
  int kind, nx, ny, nz, nrhs;
  bool operator<(const RowKey& o) const {
    return std::tie(kind, nx, ny, nz, nrhs) < std::tie(o.kind, o.nx, o.ny, o.nz, o.nrhs);
  }
};
std::mutex g_row_mu;
std::map<RowKey, int> g_row_tune;
std::atomic<int> g_row_forced{0};

bool row_no_tune() {
  static const bool v = std::getenv("HELM_NO_TUNE") != nullptr;
  return v;
}

bool row_untuned(const RowKey& key) {
  if (key.nrhs < 4 || row_no_tune() || g_row_forced.load() != 0) return false;
  std::lock_guard<std::mutex> lk(g_row_mu);
  return g_row_tune.find(key) == g_row_tune.end();
}

// Schedules: 2, 4, 8 = row tiles with that many nodes per thread; MARCH | n =
// plane-marching with n nodes per thread (batches of 16 k right-hand sides).
constexpr int MARCH = 0x100;
bool march_ok(int nrhs) { return nrhs % 16 == 0; }

template <typename Launch>
int tuned_nxt(const RowKey& key, hipStream_t s, Launch&& launch) {
  if (const int f = g_row_forced.load()) return (f & MARCH) && !march_ok(key.nrhs) ? 4 : f;
  {
    std::lock_guard<std::mutex> lk(g_row_mu);
    auto it = g_row_tune.find(key);
    if (it != g_row_tune.end()) return it->second;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  if (row_no_tune() || cap != hipStreamCaptureStatusNone) return 4;
  hipEvent_t e0, e1;
  (void)locked_event_create(&e0);
  (void)locked_event_create(&e1);
  int bestn = 4;
  float best = 1e30f;
  std::vector<int> cand{2, 4, 8};
  if (march_ok(key.nrhs)) {
    cand.push_back(MARCH | 2);
    cand.push_back(MARCH | 3);
  }
  for (int nxt : cand) {
    float tot = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(e0, s);
      launch(nxt);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) tot += ms;
    }
    static const bool verbose_c = std::getenv("HELM_TUNE_VERBOSE") != nullptr;
    if (verbose_c)
      std::fprintf(stderr, "helm:   candidate %s, %d nodes per thread: %.3f ms\n",
                   (nxt & MARCH) ? "plane-marching" : "row tiles", nxt & 0xff, tot);
    if (tot < best) {
      best = tot;
      bestn = nxt;
    }
  }
  locked_event_destroy(e0);
  locked_event_destroy(e1);
  static const bool verbose = std::getenv("HELM_TUNE_VERBOSE") != nullptr;
  if (verbose)
    std::fprintf(stderr, "helm: %s tuned (%dx%dx%d, %d rhs): %s, %d nodes per thread, %.3f ms\n",
                 key.kind ? "coarse product" : "stencil", key.nx, key.ny, key.nz, key.nrhs,
                 (bestn & MARCH) ? "plane-marching" : "row tiles", bestn & 0xff, best);
  std::lock_guard<std::mutex> lk(g_row_mu);
  g_row_tune[key] = bestn;
  return bestn;
}

template <int NXT, int RW>
void launch_march_t(const OpDev& op, int nx, int ny, int nz, const z64* E, int nrhs, const z64* x, z64* y,
                    const z64* b, hipStream_t s) {
  hipLaunchKernelGGL((k_march<NXT, RW>), dim3(march_tiles<NXT, RW>(nx, ny, nz), (unsigned)(nrhs / RW)), dim3(256), 0,
                     s, op, nx, ny, nz, E, nrhs, x, y, b);
}
// plane-marching product with n nodes per thread (2 or 3); nrhs a multiple of 16
void launch_march(int n, const OpDev& op, int nx, int ny, int nz, const z64* E, int nrhs, const z64* x, z64* y,
                  const z64* b, hipStream_t s) {
  if (nrhs % 32 == 0) {
    if (n == 2) launch_march_t<2, 32>(op, nx, ny, nz, E, nrhs, x, y, b, s);
    else launch_march_t<3, 32>(op, nx, ny, nz, E, nrhs, x, y, b, s);
  } else {
    if (n == 2) launch_march_t<2, 16>(op, nx, ny, nz, E, nrhs, x, y, b, s);
    else launch_march_t<3, 16>(op, nx, ny, nz, E, nrhs, x, y, b, s);
  }
}
}  // namespace

bool stencil_untuned(const OpDev& op, int nrhs) { return row_untuned({0, op.nx, op.ny, op.nz, nrhs}); }
bool coarse_spmv_untuned(int ncx, int ncy, int ncz, int nrhs) { return row_untuned({1, ncx, ncy, ncz, nrhs}); }
bool set_row_tiling(int nxt) {
  if (nxt != 0 && nxt != 2 && nxt != 4 && nxt != 8 && nxt != (MARCH | 2) && nxt != (MARCH | 3)) return false;
  g_row_forced.store(nxt);
  return true;
}

static void stencil_dispatch(const OpDev& op, int nrhs, const z64* x, z64* y, const z64* b, hipStream_t s) {
  {  // x read and y written once, b read once for a residual, the node values s k^2 and the stored row
     // diagonals once; 27 complex products
    const double n = (double)op.nx * op.ny * op.nz;
    account(16.0 * n * nrhs * (b ? 3 : 2) + 32.0 * n, 216.0 * n * nrhs);
  }
  if (nrhs >= 4) {
    const dim3 grid(row_tiles(op.nx, op.ny, op.nz));
    auto launch = [&](int nxt) {
      if (nxt & MARCH) launch_march(nxt & 0xff, op, op.nx, op.ny, op.nz, nullptr, nrhs, x, y, b, s);
      else if (nxt == 2) hipLaunchKernelGGL(k_stencil_rows<2>, grid, dim3(256), 0, s, op, nrhs, x, y, b);
      else if (nxt == 8) hipLaunchKernelGGL(k_stencil_rows<8>, grid, dim3(256), 0, s, op, nrhs, x, y, b);
      else hipLaunchKernelGGL(k_stencil_rows<4>, grid, dim3(256), 0, s, op, nrhs, x, y, b);
    };
    launch(tuned_nxt({0, op.nx, op.ny, op.nz, nrhs}, s, launch));
    return;
  }
  const long long n = (long long)op.nx * op.ny * op.nz;
  const int nb = nrhs >= 256 ? 1 : (nrhs >= 4 ? 256 / nrhs : 64);
  hipLaunchKernelGGL(k_stencil2, dim3((unsigned)ceil_div(n, nb)), dim3(256), sizeof(z64) * 27 * nb, s, op, nrhs, x,
                     y, b);
}

void launch_stencil(const OpDev& op, int nrhs, const z64* x, z64* y, hipStream_t s) {
  stencil_dispatch(op, nrhs, x, y, nullptr, s);
}

void launch_residual(const OpDev& op, int nrhs, const z64* b, const z64* x, z64* y, hipStream_t s) {
  stencil_dispatch(op, nrhs, x, y, b, s);
}

void launch_build_E(const OpDev& op, int ncx, int ncy, int ncz, z64* E, hipStream_t s) {
  const long long nc = (long long)ncx * ncy * ncz;
  hipLaunchKernelGGL(k_build_E, dim3((unsigned)ceil_div(nc, BUILD_E_BLOCK)), dim3(BUILD_E_BLOCK), 0, s, op, ncx, ncy,
                     ncz, E);
}

void launch_coarse_spmv(int ncx, int ncy, int ncz, const z64* E, int nrhs, const z64* x, z64* y,
                        hipStream_t s) {
  {  // E once (27 coefficients per node), x read and y written once
    const double nc = (double)ncx * ncy * ncz;
    account(nc * (27.0 * 16 + 32.0 * nrhs), 216.0 * nc * nrhs);
  }
  if (nrhs >= 4) {
    const dim3 grid(row_tiles(ncx, ncy, ncz));
    auto launch = [&](int nxt) {
      if (nxt & MARCH) launch_march(nxt & 0xff, OpDev{}, ncx, ncy, ncz, E, nrhs, x, y, nullptr, s);
      else if (nxt == 2) hipLaunchKernelGGL(k_coarse_spmv_rows<2>, grid, dim3(256), 0, s, ncx, ncy, ncz, E, nrhs, x, y);
      else if (nxt == 8) hipLaunchKernelGGL(k_coarse_spmv_rows<8>, grid, dim3(256), 0, s, ncx, ncy, ncz, E, nrhs, x, y);
      else hipLaunchKernelGGL(k_coarse_spmv_rows<4>, grid, dim3(256), 0, s, ncx, ncy, ncz, E, nrhs, x, y);
    };
    launch(tuned_nxt({1, ncx, ncy, ncz, nrhs}, s, launch));
    return;
  }
  const long long nc = (long long)ncx * ncy * ncz;
  hipLaunchKernelGGL(k_coarse_spmv2, dim3((unsigned)ceil_div(nc * nrhs, 256)), dim3(256), 0, s, ncx, ncy, ncz, E, nrhs,
                     x, y);
}

void launch_restrict(int nx, int ny, int nz, int nrhs, const z64* r, z64* c, hipStream_t s) {
  const long long nc = (long long)((nx + 1) / 2) * ((ny + 1) / 2) * ((nz + 1) / 2);
  account(16.0 * ((double)nx * ny * nz + nc) * nrhs, 2.0 * 27 * nc * nrhs);
  const dim3 grid((unsigned)ceil_div((long long)((nx + 1) / 2) * nrhs, 256), (ny + 1) / 2, (nz + 1) / 2);
  hipLaunchKernelGGL(k_restrict, grid, dim3(256), 0, s, nx, ny, nz, nrhs, r, c);
}

void launch_prolong(int nx, int ny, int nz, int nrhs, const z64* c, z64* q, hipStream_t s) {
  const long long n = (long long)nx * ny * nz;
  account(16.0 * (n + (double)((nx + 1) / 2) * ((ny + 1) / 2) * ((nz + 1) / 2)) * nrhs, 2.0 * 8 * n * nrhs);
  hipLaunchKernelGGL(k_prolong, dim3((unsigned)ceil_div((long long)nx * nrhs, 256), ny, nz), dim3(256), 0, s, nx, ny, nz,
                     nrhs, c, q);
}
