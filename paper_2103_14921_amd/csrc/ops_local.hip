// Local problems of the ORAS preconditioner (eq. oras): assembly of the
// subdomain operators A_i with absorbing interfaces, their block-tridiagonal
// (plane-by-plane) factorisation, and the batched local solves.
//
// A_i is block tridiagonal over the z-planes of its box: diagonal blocks D_k
// (in-plane 9-point couplings, b x b with b = ex*ey), sub-diagonal L_k (plane k
// to k-1) and super-diagonal U_k (plane k to k+1), each 9 entries per row.
// Block LU: S_0 = D_0, S_k = D_k - L_k S_{k-1}^{-1} U_{k-1}.  The dense Schur
// blocks are inverted explicitly (blocked Gauss-Jordan with partial pivoting
// inside each block), so that both sweeps are dense products:
//   forward   y_k = S_k^{-1} (f_k - L_k y_{k-1})
//   backward  x_k = y_k - S_k^{-1} (U_k x_{k+1}),  x_{ez-1} = y_{ez-1}.
// Absorbing interface (Robin fold): for a box node l with a grid neighbour j
// outside the box, A_i[l, l] += A[l, j] (1 + i k_l h) -- the ghost value is
// replaced by the first-order outgoing condition u_j ~ (1 + i k h) u_l.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.h"
#include "mfma.h"
#include "stencil_row.h"

namespace {

__global__ void __launch_bounds__(256) k_local_fine(OpDev op, const Sub* __restrict__ subs, const z64* __restrict__ c,
                             double omega, double h, int robin, z64* __restrict__ aloc) {
  const Sub sb = subs[blockIdx.y];
  const long long nl = (long long)sb.ex * sb.ey * sb.ez;
  z64 row[27];
  for (long long l = blockIdx.x * (long long)blockDim.x + threadIdx.x; l < nl;
       l += (long long)gridDim.x * blockDim.x) {
    const int lx = (int)(l % sb.ex), ly = (int)((l / sb.ex) % sb.ey), lz = (int)(l / ((long long)sb.ex * sb.ey));
    const int gx = sb.elo[0] + lx, gy = sb.elo[1] + ly, gz = sb.elo[2] + lz;
    fine_row(op, gx, gy, gz, row);
    z64 fold = mk(0.0, 0.0);
    z64* out = aloc + (sb.node_off + l) * 27;
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      if (o == 13) continue;
      const int jx = gx + o % 3 - 1, jy = gy + (o / 3) % 3 - 1, jz = gz + o / 9 - 1;
      const bool in_box = jx >= sb.elo[0] && jx < sb.ehi[0] && jy >= sb.elo[1] && jy < sb.ehi[1] &&
                          jz >= sb.elo[2] && jz < sb.ehi[2];
      if (in_box) {
        out[o] = row[o];
      } else {
        fold += row[o];  // zero for ghost neighbours outside the grid
        out[o] = mk(0.0, 0.0);
      }
    }
    z64 d = row[13];
    if (robin) {
      const z64 k = cdiv(mk(omega, 0.0), c[gx + (long long)op.nx * (gy + (long long)op.ny * gz)]);
      d += fold * mk(1.0 - k.im * h, k.re * h);
    }
    out[13] = d;
  }
}

__global__ void k_local_coarse(int ncx, int ncy, int ncz, const z64* __restrict__ E, const Sub* __restrict__ subs,
                               const z64* __restrict__ cf, int nx, int ny, double omega, double hc, int robin,
                               z64* __restrict__ aloc) {
  const Sub sb = subs[blockIdx.y];
  const long long nl = (long long)sb.ex * sb.ey * sb.ez;
  for (long long l = blockIdx.x * (long long)blockDim.x + threadIdx.x; l < nl;
       l += (long long)gridDim.x * blockDim.x) {
    const int lx = (int)(l % sb.ex), ly = (int)((l / sb.ex) % sb.ey), lz = (int)(l / ((long long)sb.ex * sb.ey));
    const int gx = sb.elo[0] + lx, gy = sb.elo[1] + ly, gz = sb.elo[2] + lz;
    const z64* row = E + (gx + (long long)ncx * (gy + (long long)ncy * gz)) * 27;
    z64 fold = mk(0.0, 0.0);
    z64* out = aloc + (sb.node_off + l) * 27;
    for (int o = 0; o < 27; ++o) {
      if (o == 13) continue;
      const int jx = gx + o % 3 - 1, jy = gy + (o / 3) % 3 - 1, jz = gz + o / 9 - 1;
      const bool in_box = jx >= sb.elo[0] && jx < sb.ehi[0] && jy >= sb.elo[1] && jy < sb.ehi[1] &&
                          jz >= sb.elo[2] && jz < sb.ehi[2];
      const bool in_grid = jx >= 0 && jx < ncx && jy >= 0 && jy < ncy && jz >= 0 && jz < ncz;
      if (in_box) {
        out[o] = row[o];
      } else {
        if (in_grid) fold += row[o];
        out[o] = mk(0.0, 0.0);
      }
    }
    z64 d = row[13];
    if (robin) {
      // k of the co-located fine node (2I, 2J, 2K), coarse spacing hc = 2h
      const z64 k = cdiv(mk(omega, 0.0), cf[2 * gx + (long long)nx * (2 * gy + (long long)ny * 2 * gz)]);
      d += fold * mk(1.0 - k.im * hc, k.re * hc);
    }
    out[13] = d;
  }
}

// W = Sinv_{k-1} U_{k-1}:  W[p][q] = sum_{a in N(q)} Sinv[p][a] U[a][q],  U[a][q] = A_i[(k-1,a),(k,q)]
// A workgroup owns 64 columns q and 32 rows p of one box: the nine coupling
// values U[a][q] of its columns (and their plane indices a) are staged in LDS
// once, instead of being gathered from the 27-wide local rows by every
// output; out-of-plane neighbours get a zero coupling and keep the term order.
constexpr int SW_TQ = 64, SW_TP = 32;
template <typename T>
__global__ void __launch_bounds__(256) k_schur_W(const Sub* __restrict__ subs, int k, int bpmax,
                                                 const z64* __restrict__ aloc, const cpx<T>* __restrict__ sinv,
                                                 cpx<T>* __restrict__ W) {
  const Sub sb = subs[blockIdx.z];
  const int b = sb.b;
  const int q0 = blockIdx.x * SW_TQ, p0 = blockIdx.y * SW_TP;
  if (k < 1 || k >= sb.ez || q0 >= b || p0 >= b) return;  // uniform over the workgroup
  __shared__ cpx<T> uc[SW_TQ][9];
  __shared__ int ua[SW_TQ][9];
  for (int e = threadIdx.x; e < SW_TQ * 9; e += blockDim.x) {
    const int ql = e / 9, d = e % 9, dy = d / 3 - 1, dx = d % 3 - 1;
    const int q = q0 + ql;
    cpx<T> u = mk<T>(0, 0);
    int a = 0;
    if (q < b) {
      const int ax = q % sb.ex + dx, ay = q / sb.ex + dy;
      if (ax >= 0 && ax < sb.ex && ay >= 0 && ay < sb.ey) {
        a = ax + sb.ex * ay;
        // offset from a (plane k-1) to q (plane k): (-dx, -dy, +1)
        u = ccast<T>(aloc[(sb.node_off + (long long)(k - 1) * b + a) * 27 + 18 + (1 - dy) * 3 + (1 - dx)]);
      }
    }
    uc[ql][d] = u;
    ua[ql][d] = a;
  }
  __syncthreads();
  const int ql = threadIdx.x % SW_TQ, q = q0 + ql;
  if (q >= b) return;
  const cpx<T>* Sb = sinv + sb.mat_off + (long long)(k - 1) * sb.bp * sb.bp;
  cpx<T>* Wb = W + (long long)blockIdx.z * bpmax * bpmax;
  const int pend = min(p0 + SW_TP, b);
  for (int p = p0 + threadIdx.x / SW_TQ; p < pend; p += 256 / SW_TQ) {
    const cpx<T>* Sp = Sb + (long long)p * sb.bp;
    cpx<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int d = 0; d < 9; ++d) cfma(acc, Sp[ua[ql][d]], uc[ql][d]);
    Wb[(long long)p * sb.bp + q] = acc;
  }
}

// S[p][q] = D_k[p][q] - sum_{c in N(p)} L_k[p][c] W[c][q]  (no L term at k = 0); padding zero
template <typename T>
__global__ void k_schur_S(const Sub* __restrict__ subs, int k, int bpmax, const z64* __restrict__ aloc,
                          const cpx<T>* __restrict__ W, cpx<T>* __restrict__ S) {
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const int b = sb.b, bp = sb.bp;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)bp * bp) return;
  const int p = (int)(t / bp), q = (int)(t % bp);
  cpx<T>* out = S + (long long)s * bpmax * bpmax + (long long)p * bp + q;
  if (p >= b || q >= b) {
    *out = mk<T>(0, 0);
    return;
  }
  const int px = p % sb.ex, py = p / sb.ex, qx = q % sb.ex, qy = q / sb.ex;
  const z64* rowp = aloc + (sb.node_off + (long long)k * b + p) * 27;
  cpx<T> acc = mk<T>(0, 0);
  const int dx = qx - px, dy = qy - py;
  if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) acc = ccast<T>(rowp[9 + (dy + 1) * 3 + (dx + 1)]);
  if (k >= 1) {
    const cpx<T>* Wb = W + (long long)s * bpmax * bpmax;
    for (int ey = -1; ey <= 1; ++ey) {
      const int cy = py + ey;
      if (cy < 0 || cy >= sb.ey) continue;
      for (int ex = -1; ex <= 1; ++ex) {
        const int cx = px + ex;
        if (cx < 0 || cx >= sb.ex) continue;
        const int cc = cx + sb.ex * cy;
        cfms(acc, ccast<T>(rowp[(ey + 1) * 3 + (ex + 1)]), Wb[(long long)cc * bp + q]);
      }
    }
  }
  *out = acc;
}

template <typename T>
__device__ __forceinline__ T cabs1(cpx<T> a) {
  return fabs(a.re) + fabs(a.im);
}

// Gauss-Jordan on the panel of columns [j0, j0+NB) of S (all b rows), partial
// pivoting over rows >= j.  Row i of the panel lives in thread i % 256, slot i / 256.
template <typename T, int NB, int R>
__global__ void __launch_bounds__(256) k_gj_panel(const Sub* __restrict__ subs, int k, int j0, int bpmax,
                                                  cpx<T>* __restrict__ S, int* __restrict__ piv,
                                                  int* __restrict__ err) {
  const int s = blockIdx.x;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const int b = sb.b, bp = sb.bp;
  if (j0 >= b) return;
  const int nbw = min(NB, b - j0);
  cpx<T>* A = S + (long long)s * bpmax * bpmax;
  const int tid = threadIdx.x;
  __shared__ cpx<T> rowA[NB], rowB[NB], prow[NB];
  __shared__ T rv[4];
  __shared__ int ri[4];
  cpx<T> P[R][NB];
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    const int i = tid + 256 * rr;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      P[rr][c] = (i < b && c < nbw) ? A[(long long)i * bp + j0 + c] : mk<T>(0, 0);
  }
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) {
    if (jj >= nbw) continue;  // uniform; a constant trip count keeps P in registers
    const int j = j0 + jj;
    // pivot search: largest |re|+|im| over rows i >= j, ties to the smallest index
    T best = (T)-1;
    int bi = 0x7fffffff;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int i = tid + 256 * rr;
      if (i >= j && i < b) {
        const T m = cabs1(P[rr][jj]);
        if (m > best || (m == best && i < bi)) { best = m; bi = i; }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const T ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if ((tid & 63) == 0) { rv[tid >> 6] = best; ri[tid >> 6] = bi; }
    __syncthreads();
    if (tid == 0) {
      T bb = rv[0];
      int ii = ri[0];
      for (int w = 1; w < 4; ++w)
        if (rv[w] > bb || (rv[w] == bb && ri[w] < ii)) { bb = rv[w]; ii = ri[w]; }
      ri[0] = ii;
      rv[0] = bb;
      piv[(long long)s * bpmax + j] = ii;
      if (!(bb > (T)0)) atomicOr(err, 1);
    }
    __syncthreads();
    const int p = ri[0];
    const bool sing = !(rv[0] > (T)0);
    // swap rows j and p of the panel
    if (p != j) {
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int i = tid + 256 * rr;
        if (i == j) {
#pragma unroll
          for (int c = 0; c < NB; ++c) rowA[c] = P[rr][c];
        }
        if (i == p) {
#pragma unroll
          for (int c = 0; c < NB; ++c) rowB[c] = P[rr][c];
        }
      }
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int i = tid + 256 * rr;
        if (i == j) {
#pragma unroll
          for (int c = 0; c < NB; ++c) P[rr][c] = rowB[c];
        }
        if (i == p) {
#pragma unroll
          for (int c = 0; c < NB; ++c) P[rr][c] = rowA[c];
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
      if (tid + 256 * rr == j) {
#pragma unroll
        for (int c = 0; c < NB; ++c) prow[c] = P[rr][c];
      }
    __syncthreads();
    const cpx<T> inv = sing ? mk<T>(1, 0) : cinv(prow[jj]);
    cpx<T> pr[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) pr[c] = (c == jj) ? inv : prow[c] * inv;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int i = tid + 256 * rr;
      if (i >= b) continue;
      if (i == j) {
#pragma unroll
        for (int c = 0; c < NB; ++c) P[rr][c] = pr[c];
      } else {
        const cpx<T> f = P[rr][jj];
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c != jj) cfms(P[rr][c], f, pr[c]);
        P[rr][jj] = -(f * inv);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    const int i = tid + 256 * rr;
    if (i < b)
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) A[(long long)i * bp + j0 + c] = P[rr][c];
  }
}

// Apply the panel's row interchanges to the columns outside the panel and copy
// the (interchanged) pivot rows to Rbuf[s][jj][c].
template <typename T, int NB>
__global__ void k_gj_swap(const Sub* __restrict__ subs, int k, int j0, int bpmax, cpx<T>* __restrict__ S,
                          const int* __restrict__ piv, cpx<T>* __restrict__ Rbuf) {
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const int b = sb.b, bp = sb.bp;
  if (j0 >= b) return;
  const int nbw = min(NB, b - j0);
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b || (c >= j0 && c < j0 + nbw)) return;
  cpx<T>* A = S + (long long)s * bpmax * bpmax;
  for (int jj = 0; jj < nbw; ++jj) {
    const int j = j0 + jj;
    const int p = piv[(long long)s * bpmax + j];
    if (p != j) {
      const cpx<T> t = A[(long long)j * bp + c];
      A[(long long)j * bp + c] = A[(long long)p * bp + c];
      A[(long long)p * bp + c] = t;
    }
  }
  for (int jj = 0; jj < nbw; ++jj)
    Rbuf[((long long)s * NB + jj) * bpmax + c] = A[(long long)(j0 + jj) * bp + c];
}

// Pivot rows of a block of OB Gauss-Jordan columns [J0, J0 + OB), as they stand
// after the block's row interchanges (the columns outside the block are only
// interchanged while the block is processed), for the block's deferred update.
constexpr int GJ_OB = 64;

template <typename T>
__global__ void k_gj_rows(const Sub* __restrict__ subs, int k, int J0, int bpmax, const cpx<T>* __restrict__ S,
                          cpx<T>* __restrict__ R64) {
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const int b = sb.b, bp = sb.bp;
  if (J0 >= b) return;
  const int nbw = min(GJ_OB, b - J0);
  const cpx<T>* A = S + (long long)s * bpmax * bpmax;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nbw * b; e += gridDim.x * blockDim.x) {
    const int jj = e / b, c = e % b;
    R64[((long long)s * GJ_OB + jj) * bpmax + c] = A[(long long)(J0 + jj) * bp + c];
  }
}

// Deferred update of the columns outside the processed block on matrix cores:
// A[i][c] = (i in block rows ? 0 : A[i][c]) + sum_jj A[i][J0 + jj] R64[jj][c],
// a rank-OB complex product.  A workgroup owns a 64 x 64 tile of one box's
// matrix; its R64 rows are staged in LDS, each of the four waves forms 16 rows
// with the planar complex scheme (real and imaginary accumulators, four real
// MFMAs per 16x16x4 step).
template <typename T>
__global__ void __launch_bounds__(256) k_gj_outer(const Sub* __restrict__ subs, int k, int J0, int bpmax,
                                                  cpx<T>* __restrict__ S, const cpx<T>* __restrict__ R64) {
  using V4 = typename Mfma<T>::v4;
  constexpr int RW = 64 + (sizeof(T) == 4 ? 4 : 2);  // padded LDS row
  __shared__ cpx<T> Rs[GJ_OB][RW];
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const int b = sb.b, bp = sb.bp;
  if (J0 >= b) return;
  const int nbw = min(GJ_OB, b - J0);
  const int ntc = (b + 63) / 64;
  const int i0 = (blockIdx.x / ntc) * 64, c0 = (blockIdx.x % ntc) * 64;
  if (i0 >= b) return;
  if (c0 >= J0 && c0 + 64 <= J0 + nbw) return;  // every column of the tile is in the block
  cpx<T>* A = S + (long long)s * bpmax * bpmax;
  for (int e = threadIdx.x; e < GJ_OB * 64; e += 256) {
    const int kk = e / 64, cc = e % 64;
    Rs[kk][cc] = (kk < nbw && c0 + cc < b) ? R64[((long long)s * GJ_OB + kk) * bpmax + c0 + cc] : mk<T>(0, 0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lrow = lane & 15, lg = lane >> 4;
  const int row = i0 + 16 * wave + lrow;
  const cpx<T>* Arow = A + (long long)min(row, b - 1) * bp + J0;  // clamped: rows past b contribute nothing stored
  V4 acc[4][2];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt][0] = acc[nt][1] = V4{0, 0, 0, 0};
  for (int kc = 0; kc < nbw; kc += 16) {
    cpx<T> av[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int kk = kc + 4 * lg + t;
      av[t] = kk < nbw ? Arow[kk] : mk<T>(0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T are = av[t].re, aim = av[t].im, naim = -aim;
      const int kk = kc + 4 * lg + t;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const cpx<T> tv = Rs[kk][nt * 16 + lrow];
        acc[nt][0] = Mfma<T>::op(are, tv.re, acc[nt][0]);
        acc[nt][1] = Mfma<T>::op(are, tv.im, acc[nt][1]);
        acc[nt][0] = Mfma<T>::op(naim, tv.im, acc[nt][0]);
        acc[nt][1] = Mfma<T>::op(aim, tv.re, acc[nt][1]);
      }
    }
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 16 * wave + Mfma<T>::row(lg, v), c = c0 + nt * 16 + lrow;
      if (i >= b || c >= b || (c >= J0 && c < J0 + nbw)) continue;
      cpx<T>* a = A + (long long)i * bp + c;
      const cpx<T> old = (i >= J0 && i < J0 + nbw) ? mk<T>(0, 0) : *a;
      *a = mk<T>(old.re + acc[nt][0][v], old.im + acc[nt][1][v]);
    }
}

// The panel's deferred update inside its block on matrix cores:
// A[i][c] = (i in panel rows ? 0 : A[i][c]) + sum_jj A[i][j0 + jj] R[jj][c]
// for the block's columns c in [J0, J0 + OB) outside the panel, a rank-NB
// complex product (R = the interchanged pivot rows in Rbuf[s][jj][c]).  A
// workgroup owns 64 rows of one box's block; the R rows are staged in LDS and
// each of the four waves forms 16 rows with the planar complex scheme.
template <typename T, int NB>
__global__ void __launch_bounds__(256) k_gj_inner(const Sub* __restrict__ subs, int k, int j0, int J0, int bpmax,
                                                  cpx<T>* __restrict__ S, const cpx<T>* __restrict__ Rbuf) {
  using V4 = typename Mfma<T>::v4;
  constexpr int RW = 64 + (sizeof(T) == 4 ? 4 : 2);  // padded LDS row
  __shared__ cpx<T> Rs[NB][RW];
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const int b = sb.b, bp = sb.bp;
  if (j0 >= b) return;
  const int nbw = min(NB, b - j0);
  const int i0 = blockIdx.x * 64;
  if (i0 >= b) return;
  cpx<T>* A = S + (long long)s * bpmax * bpmax;
  for (int e = threadIdx.x; e < NB * 64; e += 256) {
    const int kk = e / 64, cc = e % 64;
    Rs[kk][cc] = (kk < nbw && J0 + cc < b) ? Rbuf[((long long)s * NB + kk) * bpmax + J0 + cc] : mk<T>(0, 0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lrow = lane & 15, lg = lane >> 4;
  const int row = i0 + 16 * wave + lrow;
  const cpx<T>* Arow = A + (long long)min(row, b - 1) * bp + j0;  // clamped: rows past b contribute nothing stored
  V4 acc[4][2];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt][0] = acc[nt][1] = V4{0, 0, 0, 0};
#pragma unroll
  for (int kc = 0; kc < NB; kc += 16) {
    cpx<T> av[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int kk = kc + 4 * lg + t;
      av[t] = kk < nbw ? Arow[kk] : mk<T>(0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T are = av[t].re, aim = av[t].im, naim = -aim;
      const int kk = min(kc + 4 * lg + t, NB - 1);  // past the panel: av is zero
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const cpx<T> tv = Rs[kk][nt * 16 + lrow];
        acc[nt][0] = Mfma<T>::op(are, tv.re, acc[nt][0]);
        acc[nt][1] = Mfma<T>::op(are, tv.im, acc[nt][1]);
        acc[nt][0] = Mfma<T>::op(naim, tv.im, acc[nt][0]);
        acc[nt][1] = Mfma<T>::op(aim, tv.re, acc[nt][1]);
      }
    }
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 16 * wave + Mfma<T>::row(lg, v), c = J0 + nt * 16 + lrow;
      if (i >= b || c >= b || (c >= j0 && c < j0 + nbw)) continue;
      cpx<T>* a = A + (long long)i * bp + c;
      const cpx<T> old = (i >= j0 && i < j0 + nbw) ? mk<T>(0, 0) : *a;
      *a = mk<T>(old.re + acc[nt][0][v], old.im + acc[nt][1][v]);
    }
}

// Column permutation that undoes the row interchanges: apply swaps (j, piv[j])
// for j = b-1 .. 0 to an identity array.
__global__ void k_gj_perm(const Sub* __restrict__ subs, int nsub, int k, int bpmax, const int* __restrict__ piv,
                          int* __restrict__ perm) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsub) return;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  int* pm = perm + (long long)s * bpmax;
  for (int c = 0; c < sb.b; ++c) pm[c] = c;
  for (int j = sb.b - 1; j >= 0; --j) {
    const int p = piv[(long long)s * bpmax + j];
    const int t = pm[j];
    pm[j] = pm[p];
    pm[p] = t;
  }
}

template <typename T>
__global__ void k_gj_final(const Sub* __restrict__ subs, int k, int bpmax, const cpx<T>* __restrict__ S,
                           const int* __restrict__ perm, cpx<T>* __restrict__ sinv) {
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const int b = sb.b, bp = sb.bp;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)bp * bp) return;
  const int i = (int)(t / bp), c = (int)(t % bp);
  cpx<T> v = mk<T>(0, 0);
  if (i < b && c < b) v = S[(long long)s * bpmax * bpmax + (long long)i * bp + perm[(long long)s * bpmax + c]];
  sinv[sb.mat_off + (long long)k * bp * bp + (long long)i * bp + c] = v;
}

// ---- sweeps -----------------------------------------------------------------

// tbuf[s][p][r] = f_k[p][r] - sum_{c in N(p)} L_k[p][c] y_{k-1}[c][r], f = R_i u
template <typename T>
__global__ void k_fwd_rhs(const Sub* __restrict__ subs, int k, int bpmax, const cpx<T>* __restrict__ cpl,
                          int nrhs, const z64* __restrict__ u, int gnx, int gny, const cpx<T>* __restrict__ yloc,
                          cpx<T>* __restrict__ tbuf) {
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)sb.bp * nrhs) return;
  const int p = (int)(t / nrhs), r = (int)(t % nrhs);
  cpx<T>* out = tbuf + ((long long)s * bpmax + p) * nrhs + r;
  if (p >= sb.b) {
    *out = mk<T>(0, 0);
    return;
  }
  const int px = p % sb.ex, py = p / sb.ex;
  const long long g = (sb.elo[0] + px) + (long long)gnx * ((sb.elo[1] + py) + (long long)gny * (sb.elo[2] + k));
  cpx<T> v = ccast<T>(u[g * nrhs + r]);
  if (k >= 1) {
    const cpx<T>* rowp = cpl + (sb.node_off + (long long)k * sb.b + p) * 18;
    const cpx<T>* yprev = yloc + (sb.vec_off + (long long)(k - 1) * sb.bp) * nrhs + r;
    for (int dy = -1; dy <= 1; ++dy) {
      const int cy = py + dy;
      if (cy < 0 || cy >= sb.ey) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int cx = px + dx;
        if (cx < 0 || cx >= sb.ex) continue;
        cfms(v, rowp[(dy + 1) * 3 + (dx + 1)], yprev[(long long)(cx + sb.ex * cy) * nrhs]);
      }
    }
  }
  *out = v;
}

// tbuf[s][p][r] = sum_{c in N(p)} U_k[p][c] x_{k+1}[c][r],  k = ez - 2 - step
template <typename T>
__global__ void k_bwd_rhs(const Sub* __restrict__ subs, int step, int bpmax, const cpx<T>* __restrict__ cpl,
                          int nrhs, const cpx<T>* __restrict__ yloc, cpx<T>* __restrict__ tbuf) {
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  const int k = sb.ez - 2 - step;
  if (k < 0) return;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)sb.bp * nrhs) return;
  const int p = (int)(t / nrhs), r = (int)(t % nrhs);
  cpx<T>* out = tbuf + ((long long)s * bpmax + p) * nrhs + r;
  if (p >= sb.b) {
    *out = mk<T>(0, 0);
    return;
  }
  const int px = p % sb.ex, py = p / sb.ex;
  const cpx<T>* rowp = cpl + (sb.node_off + (long long)k * sb.b + p) * 18 + 9;
  const cpx<T>* xnext = yloc + (sb.vec_off + (long long)(k + 1) * sb.bp) * nrhs + r;
  cpx<T> v = mk<T>(0, 0);
  for (int dy = -1; dy <= 1; ++dy) {
    const int cy = py + dy;
    if (cy < 0 || cy >= sb.ey) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      const int cx = px + dx;
      if (cx < 0 || cx >= sb.ex) continue;
      cfma(v, rowp[(dy + 1) * 3 + (dx + 1)], xnext[(long long)(cx + sb.ex * cy) * nrhs]);
    }
  }
  *out = v;
}

// Dense plane product on all subdomains: acc = Sinv_k tbuf;
// forward (bwd == 0, k = step): y_k = acc;  backward (k = ez-2-step): y_k -= acc.
template <typename T, int NR>
__global__ void __launch_bounds__(256) k_plane_gemm(const Sub* __restrict__ subs, int step, int bwd, int bpmax,
                                                    const cpx<T>* __restrict__ sinv, int nrhs,
                                                    const cpx<T>* __restrict__ tbuf, cpx<T>* __restrict__ yloc) {
  const int s = blockIdx.y;
  const Sub sb = subs[s];
  const int k = bwd ? sb.ez - 2 - step : step;
  if (k < 0 || k >= sb.ez) return;
  const int nch = nrhs / NR;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)sb.bp * nch) return;
  const int p = (int)(t / nch), r0 = (int)(t % nch) * NR;
  const cpx<T>* Sp = sinv + sb.mat_off + (long long)k * sb.bp * sb.bp + (long long)p * sb.bp;
  const cpx<T>* tb = tbuf + (long long)s * bpmax * nrhs + r0;
  cpx<T> acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = mk<T>(0, 0);
  for (int q = 0; q < sb.b; ++q) {
    const cpx<T> a = Sp[q];
#pragma unroll
    for (int r = 0; r < NR; ++r) cfma(acc[r], a, tb[(long long)q * nrhs + r]);
  }
  cpx<T>* y = yloc + (sb.vec_off + (long long)k * sb.bp + p) * nrhs + r0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (bwd) y[r] = y[r] - acc[r];
    else y[r] = acc[r];
  }
}

// z[g][r] = x_i[l][r] (+ add[g][r]) on the core nodes of every box (Boolean D_i)
template <typename T>
__global__ void k_scatter(const Sub* __restrict__ subs, int nrhs, const cpx<T>* __restrict__ yloc, int gnx, int gny,
                          z64* __restrict__ z, const z64* __restrict__ add) {
  const Sub sb = subs[blockIdx.y];
  const int cx = sb.hi[0] - sb.lo[0], cy = sb.hi[1] - sb.lo[1], cz = sb.hi[2] - sb.lo[2];
  const long long ncore = (long long)cx * cy * cz;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < ncore * nrhs;
       t += (long long)gridDim.x * blockDim.x) {
    const long long l = t / nrhs;
    const int r = (int)(t % nrhs);
    const int x = sb.lo[0] + (int)(l % cx), y = sb.lo[1] + (int)((l / cx) % cy), zz = sb.lo[2] + (int)(l / ((long long)cx * cy));
    const int lx = x - sb.elo[0], ly = y - sb.elo[1], lz = zz - sb.elo[2];
    const long long g = x + (long long)gnx * (y + (long long)gny * zz);
    z64 v = ccast<double>(yloc[(sb.vec_off + (long long)lz * sb.bp + lx + sb.ex * ly) * nrhs + r]);
    if (add) v += add[g * nrhs + r];
    z[g * nrhs + r] = v;
  }
}

}  // namespace

namespace {
// u[g(l)][r] = rl[l][r] on the nodes of one box (natural order, x fastest)
__global__ void k_box_scatter(Sub sb, int gnx, int gny, int nrhs, const z64* __restrict__ rl, z64* __restrict__ u) {
  const long long nl = (long long)sb.ex * sb.ey * sb.ez;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nl * nrhs;
       t += (long long)gridDim.x * blockDim.x) {
    const long long l = t / nrhs;
    const int r = (int)(t % nrhs);
    const int lx = (int)(l % sb.ex), ly = (int)((l / sb.ex) % sb.ey), lz = (int)(l / ((long long)sb.ex * sb.ey));
    const long long g = (sb.elo[0] + lx) + (long long)gnx * ((sb.elo[1] + ly) + (long long)gny * (sb.elo[2] + lz));
    u[g * nrhs + r] = rl[t];
  }
}
// xl[l][r] = the box's stored plane solution (plane lz, row p = l mod b)
template <typename T>
__global__ void k_box_gather(Sub sb, int nrhs, const cpx<T>* __restrict__ yloc, z64* __restrict__ xl) {
  const long long nl = (long long)sb.b * sb.ez;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nl * nrhs;
       t += (long long)gridDim.x * blockDim.x) {
    const long long l = t / nrhs;
    const int r = (int)(t % nrhs);
    const long long lz = l / sb.b, p = l % sb.b;
    xl[t] = ccast<double>(yloc[(sb.vec_off + lz * sb.bp + p) * nrhs + r]);
  }
}
}  // namespace

void launch_box_scatter(const Sub& sb, int gnx, int gny, int nrhs, const z64* rl, z64* u, hipStream_t s) {
  hipLaunchKernelGGL(k_box_scatter, dim3(1024), dim3(256), 0, s, sb, gnx, gny, nrhs, rl, u);
}
template <typename T>
void launch_box_gather(const Sub& sb, int nrhs, const cpx<T>* yloc, z64* xl, hipStream_t s) {
  hipLaunchKernelGGL(k_box_gather<T>, dim3(1024), dim3(256), 0, s, sb, nrhs, yloc, xl);
}
template void launch_box_gather<float>(const Sub&, int, const c32*, z64*, hipStream_t);
template void launch_box_gather<double>(const Sub&, int, const z64*, z64*, hipStream_t);

void launch_local_fine(const OpDev& op, const Sub* subs, int nsub, long long maxnodes, const z64* c,
                       double omega, double h, int robin, z64* aloc, hipStream_t s) {
  dim3 grid((unsigned)std::min<long long>(ceil_div(maxnodes, 256), 4096), nsub);
  hipLaunchKernelGGL(k_local_fine, grid, dim3(256), 0, s, op, subs, c, omega, h, robin, aloc);
}

void launch_local_coarse(int ncx, int ncy, int ncz, const z64* E, const Sub* subs, int nsub, long long maxnodes,
                         const z64* c_fine, int nx, int ny, double omega, double hc, int robin, z64* aloc,
                         hipStream_t s) {
  dim3 grid((unsigned)std::min<long long>(ceil_div(maxnodes, 256), 4096), nsub);
  hipLaunchKernelGGL(k_local_coarse, grid, dim3(256), 0, s, ncx, ncy, ncz, E, subs, c_fine, nx, ny, omega, hc,
                     robin, aloc);
}

// Plane couplings of the local operators, in the factor precision, for the
// sweeps: per local node the nine taps to the plane below (L_k) then the nine
// to the plane above (U_k); taps that leave the box are already zero.
template <typename T>
__global__ void k_couplings(long long nodes, const z64* __restrict__ aloc, cpx<T>* __restrict__ cpl) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nodes * 18;
       i += (long long)gridDim.x * blockDim.x) {
    const long long l = i / 18;
    const int t = (int)(i % 18);
    cpl[i] = ccast<T>(aloc[l * 27 + (t < 9 ? t : t + 9)]);
  }
}

template <typename T>
void launch_couplings(long long nodes, const z64* aloc, cpx<T>* cpl, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<long long>(ceil_div(nodes * 18, 256), 65536);
  hipLaunchKernelGGL(k_couplings<T>, dim3(blocks), dim3(256), 0, s, nodes, aloc, cpl);
}
template void launch_couplings<float>(long long, const z64*, c32*, hipStream_t);
template void launch_couplings<double>(long long, const z64*, z64*, hipStream_t);

namespace {
// Blocked Gauss-Jordan inversion of the plane Schur complements: blocks of
// GJ_OB columns, each processed as NB-column panels whose deferred updates
// touch only the block; the rest of the matrix then receives the whole block's
// update in one rank-GJ_OB product on matrix cores.
template <typename T, int NB, int R>
void gj_panels(const Sub* subs, int nsub, int bpmax, int k, cpx<T>* S, cpx<T>* Rbuf, cpx<T>* R64, int* piv, int* err,
               hipStream_t s) {
  static_assert(GJ_OB % NB == 0, "panels tile the block");
  const int nt = (int)ceil_div(bpmax, 64);
  for (int J0 = 0; J0 < bpmax; J0 += GJ_OB) {
    for (int j0 = J0; j0 < J0 + GJ_OB && j0 < bpmax; j0 += NB) {
      hipLaunchKernelGGL((k_gj_panel<T, NB, R>), dim3(nsub), dim3(256), 0, s, subs, k, j0, bpmax, S, piv, err);
      hipLaunchKernelGGL((k_gj_swap<T, NB>), dim3((unsigned)ceil_div(bpmax, 256), nsub), dim3(256), 0, s, subs, k, j0,
                         bpmax, S, piv, Rbuf);
      hipLaunchKernelGGL((k_gj_inner<T, NB>), dim3((unsigned)ceil_div(bpmax, 64), nsub), dim3(256), 0, s, subs, k, j0,
                         J0, bpmax, S, Rbuf);
    }
    if (J0 + GJ_OB >= bpmax && J0 == 0) continue;  // one block covers the matrix: nothing outside it
    hipLaunchKernelGGL(k_gj_rows<T>, dim3((unsigned)ceil_div((long long)GJ_OB * bpmax, 256), nsub), dim3(256), 0, s,
                       subs, k, J0, bpmax, S, R64);
    hipLaunchKernelGGL(k_gj_outer<T>, dim3((unsigned)(nt * nt), nsub), dim3(256), 0, s, subs, k, J0, bpmax, S, R64);
  }
}
}  // namespace

namespace {
// Panel widths admissible for rows-per-thread R (the panel lives in registers,
// R x NB complex entries per thread): the first is the default.
int gj_candidates(int R, int (&nb)[2]) {
  if (R <= 2) {
    nb[0] = 16;
    nb[1] = 8;
  } else {
    nb[0] = 8;
    nb[1] = 4;
  }
  return 2;
}

// planes of up to 512 rows (R <= 2) and of up to 2048 rows (R = 4, 6, 8)
template <typename T, int NB>
void gj_small(int R, const Sub* subs, int nsub, int bpmax, int k, cpx<T>* S, cpx<T>* Rbuf, cpx<T>* R64, int* piv,
              int* err, hipStream_t s) {
  if (R <= 1) gj_panels<T, NB, 1>(subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
  else gj_panels<T, NB, 2>(subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
}
template <typename T, int NB>
void gj_large(int R, const Sub* subs, int nsub, int bpmax, int k, cpx<T>* S, cpx<T>* Rbuf, cpx<T>* R64, int* piv,
              int* err, hipStream_t s) {
  if (R <= 4) gj_panels<T, NB, 4>(subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
  else if (R <= 6) gj_panels<T, NB, 6>(subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
  else gj_panels<T, NB, 8>(subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
}

template <typename T>
void gj_dispatch(int nb, const Sub* subs, int nsub, int bpmax, int k, cpx<T>* S, cpx<T>* Rbuf, cpx<T>* R64, int* piv,
                 int* err, hipStream_t s) {
  const int R = (int)ceil_div(bpmax, 256);
  if (R <= 2) {
    if (nb == 8) gj_small<T, 8>(R, subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
    else gj_small<T, 16>(R, subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
  } else {
    if (nb == 4) gj_large<T, 4>(R, subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
    else gj_large<T, 8>(R, subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
  }
}

// Autotuned panel width of the blocked Gauss-Jordan inversion, per (precision,
// padded plane size, number of boxes): every admissible width is timed twice on
// the first plane (its factorisation is recomputed from the local rows, so
// repeating it changes nothing) and the fastest kept.
struct GjKey {
  int es, bpmax, nsub;
  bool operator<(const GjKey& o) const { return std::tie(es, bpmax, nsub) < std::tie(o.es, o.bpmax, o.nsub); }
};
std::mutex g_gj_mu;
std::map<GjKey, int> g_gj_tune;
std::atomic<int> g_gj_forced{0};
}  // namespace

bool set_lu_panel(int nb) {
  if (nb != 0 && nb != 4 && nb != 8 && nb != 16) return false;
  g_gj_forced.store(nb);
  return true;
}

namespace {
// Width for this shape: forced (where admissible), tuned, or the default.
template <typename T>
int gj_width(int bpmax, int nsub) {
  int nb[2];
  const int nc = gj_candidates((int)ceil_div(bpmax, 256), nb);
  if (const int f = g_gj_forced.load())
    for (int i = 0; i < nc; ++i)
      if (nb[i] == f) return f;
  std::lock_guard<std::mutex> lk(g_gj_mu);
  auto it = g_gj_tune.find({(int)sizeof(T), bpmax, nsub});
  return it == g_gj_tune.end() ? nb[0] : it->second;
}
}  // namespace

template <typename T>
void Factor<T>::plane(const Sub* subs, int nsub, int bpmax, int k, const z64* aloc, cpx<T>* sinv, cpx<T>* W,
                      cpx<T>* S, cpx<T>* Rbuf, cpx<T>* R64, int* piv, int* perm, int* err, hipStream_t s) {
  const long long cells = (long long)bpmax * bpmax;
  dim3 grid((unsigned)ceil_div(cells, 256), nsub);
  auto factor_with = [&](int nb) {
    if (k >= 1)
      hipLaunchKernelGGL(k_schur_W<T>, dim3((unsigned)ceil_div(bpmax, SW_TQ), (unsigned)ceil_div(bpmax, SW_TP), nsub),
                         dim3(256), 0, s, subs, k, bpmax, aloc, sinv, W);
    hipLaunchKernelGGL(k_schur_S<T>, grid, dim3(256), 0, s, subs, k, bpmax, aloc, W, S);
    gj_dispatch<T>(nb, subs, nsub, bpmax, k, S, Rbuf, R64, piv, err, s);
    hipLaunchKernelGGL(k_gj_perm, dim3((unsigned)ceil_div(nsub, 64)), dim3(64), 0, s, subs, nsub, k, bpmax, piv,
                       perm);
    hipLaunchKernelGGL(k_gj_final<T>, grid, dim3(256), 0, s, subs, k, bpmax, S, perm, sinv);
  };
  static const bool no_tune = std::getenv("HELM_NO_TUNE") != nullptr;
  const GjKey key{(int)sizeof(T), bpmax, nsub};
  bool tuned;
  {
    std::lock_guard<std::mutex> lk(g_gj_mu);
    tuned = g_gj_tune.count(key) != 0;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  if (k == 0 && !tuned && !no_tune && g_gj_forced.load() == 0 && cap == hipStreamCaptureStatusNone) {
    int nb[2];
    const int nc = gj_candidates((int)ceil_div(bpmax, 256), nb);
    hipEvent_t e0, e1;
    (void)locked_event_create(&e0);
    (void)locked_event_create(&e1);
    int best_nb = nb[0];
    float best = 1e30f;
    for (int i = 0; i < nc; ++i) {
      float tot = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0, s);
        factor_with(nb[i]);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) tot += ms;
      }
      if (tot < best) {
        best = tot;
        best_nb = nb[i];
      }
    }
    locked_event_destroy(e0);
    locked_event_destroy(e1);
    static const bool verbose = std::getenv("HELM_TUNE_VERBOSE") != nullptr;
    if (verbose)
      std::fprintf(stderr, "helm: LU panel tuned (fp%d, bp %d, %d boxes): %d columns, %.3f ms per plane\n",
                   (int)sizeof(T) * 8, bpmax, nsub, best_nb, best);
    std::lock_guard<std::mutex> lk(g_gj_mu);
    g_gj_tune[key] = best_nb;
  }
  factor_with(gj_width<T>(bpmax, nsub));
}

template <typename T>
void Factor<T>::sweep(const Sub* subs, int nsub, int bpmax, int maxez, const cpx<T>* cpl, const cpx<T>* sinv,
                      int nrhs, const z64* u, z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc,
                      cpx<T>* tbuf, hipStream_t s, bool may_tune) {
  static const bool no_fused = std::getenv("HELM_NO_FUSED") != nullptr;
  if (!no_fused && oras_fused<T>(subs, nsub, bpmax, cpl, sinv, nrhs, u, z, add, gnx, gny, yloc, tbuf, s, may_tune))
    return;
  dim3 gv((unsigned)ceil_div((long long)bpmax * nrhs, 256), nsub);
  const int nr = nrhs % 8 == 0 ? 8 : nrhs % 4 == 0 ? 4 : nrhs % 2 == 0 ? 2 : 1;
  dim3 gg((unsigned)ceil_div((long long)bpmax * (nrhs / nr), 256), nsub);
  auto gemm = [&](int step, int bwd) {
    switch (nr) {
      case 8: hipLaunchKernelGGL((k_plane_gemm<T, 8>), gg, dim3(256), 0, s, subs, step, bwd, bpmax, sinv, nrhs, tbuf, yloc); break;
      case 4: hipLaunchKernelGGL((k_plane_gemm<T, 4>), gg, dim3(256), 0, s, subs, step, bwd, bpmax, sinv, nrhs, tbuf, yloc); break;
      case 2: hipLaunchKernelGGL((k_plane_gemm<T, 2>), gg, dim3(256), 0, s, subs, step, bwd, bpmax, sinv, nrhs, tbuf, yloc); break;
      default: hipLaunchKernelGGL((k_plane_gemm<T, 1>), gg, dim3(256), 0, s, subs, step, bwd, bpmax, sinv, nrhs, tbuf, yloc); break;
    }
  };
  for (int step = 0; step < maxez; ++step) {
    hipLaunchKernelGGL(k_fwd_rhs<T>, gv, dim3(256), 0, s, subs, step, bpmax, cpl, nrhs, u, gnx, gny, yloc, tbuf);
    gemm(step, 0);
  }
  for (int step = 0; step + 1 < maxez; ++step) {
    hipLaunchKernelGGL(k_bwd_rhs<T>, gv, dim3(256), 0, s, subs, step, bpmax, cpl, nrhs, yloc, tbuf);
    gemm(step, 1);
  }
  hipLaunchKernelGGL(k_scatter<T>, dim3(1024, nsub), dim3(256), 0, s, subs, nrhs, yloc, gnx, gny, z, add);
}

template struct Factor<double>;
template struct Factor<float>;
