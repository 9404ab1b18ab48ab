// Fused local solves of the ORAS preconditioner (eq. oras) on matrix cores.
//
// One workgroup owns one subdomain and one group of RG right-hand sides and
// runs the whole block-tridiagonal solve in a single launch:
//   forward   T_k = R_i u (plane k) - L_k y_{k-1};  y_k = Sinv_k T_k
//   backward  T   = -U_k x_{k+1};                   x_k = y_k + Sinv_k T
// then scatters the core nodes of x (Boolean partition of unity), optionally
// adding a second field.  The plane vector lives in LDS; the dense products
// Sinv_k T stream Sinv_k from HBM through MFMA 16x16x4 tiles (operand lanes:
// A[l%16][l/16], B[l/16][l%16]; output rows differ between f32 and f64).
//
// Complex products on real MFMA: Sinv is stored interleaved (re, im), so each
// lane's A operand yields Re S and Im S together; the product is formed from
// real 16x16x4 steps as described at plane_product (no complex arithmetic and
// no lane-dependent operand selection inside the MFMA loop).
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "kernels.h"
#include "mfma.h"

namespace {

// Make this workgroup's global stores visible to its other waves.
__device__ __forceinline__ void wg_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Row width (in complex elements) of the plane operand in LDS.  RG >= 16 keeps
// T itself ([bp][RG], plus 4 elements of padding in complex FP32 so that the
// four lane groups of a read fall in different bank halves).  RG = 8 keeps the
// lane-ready split form [bp][16] described at plane_product.
template <typename T>
__host__ __device__ constexpr int lds_width(int rg) {
  return rg >= 16 ? rg + (sizeof(T) == 4 ? 4 : 0) : 16;
}

// The chunks of Sinv_k a wave reads, in order: its tiles mt = wave, wave +
// nwaves, ... (16 rows each), each cut into bp / 16 chunks of 16 columns.  The
// stream runs across tile boundaries, so the loads of the next tile's first
// chunks are in flight while the current tile finishes; past the end it
// repeats the last chunk (a harmless, always valid address), so every load is
// unconditional and the compiler can wait on exact counts.
template <typename T>
struct ChunkStream {
  const cpx<T>* base;  // row (wave*16 + lane%16), column 4*(lane/16) of Sk
  long long tile_step;  // elements between the wave's consecutive tiles
  int nct, ntw, tile, chunk;
  ChunkStream() = default;
  __device__ __forceinline__ ChunkStream(const cpx<T>* Sk, int bp, int wave, int nwaves, int lane) {
    const int nmt = bp >> 4;
    nct = nmt;
    ntw = wave < nmt ? (nmt - wave + nwaves - 1) / nwaves : 0;
    base = Sk + (long long)(min(wave, nmt - 1) * 16 + (lane & 15)) * bp + 4 * (lane >> 4);
    tile_step = (long long)nwaves * 16 * bp;
    tile = 0;
    chunk = 0;
  }
  __device__ __forceinline__ void next(cpx<T> (&dst)[4]) {
    const bool past = tile >= ntw;
    const cpx<T>* p = base + (past ? (long long)(ntw > 0 ? ntw - 1 : 0) * tile_step + 16 * (nct - 1)
                                   : (long long)tile * tile_step + 16 * chunk);
#pragma unroll
    for (int t = 0; t < 4; ++t) dst[t] = p[t];
    if (++chunk == nct) {
      chunk = 0;
      ++tile;
    }
  }
};

// Start a wave's chunk stream: the first PF chunks, issued before the barrier
// that publishes the plane operand.
template <typename T, int PF>
__device__ __forceinline__ ChunkStream<T> prefetch_tile(const cpx<T>* __restrict__ Sk, int bp, int wave, int nwaves,
                                                        int lane, cpx<T> (&a)[PF][4]) {
  ChunkStream<T> cs(Sk, bp, wave, nwaves, lane);
#pragma unroll
  for (int j = 0; j < PF; ++j) cs.next(a[j]);
  return cs;
}

// Rows of the wave's M-tiles of Sinv_k x T (T = plane operand in LDS): the
// wave walks its chunk stream with PF chunks in flight.  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16] of each 16x16x4 step; chunk c, step t covers
// column 16 c + 4 (l/16) + t of Sinv_k.
//
// RG >= 16 (planar): each 16-column tile of complex right-hand sides keeps a
// real and an imaginary accumulator,
//   Re C += Re S Re T - Im S Im T,   Im C += Re S Im T + Im S Re T,
// four real MFMAs per step whose B operands are read straight from T.
// RG = 8 (split): one accumulator whose columns 0..7 hold Re C and 8..15 Im C;
// with B1 = [Re T | Im T] and B2 = [-Im T | Re T],  C = Re S B1 + Im S B2.  The
// operand pair (B1, B2) of each lane is stored ready in LDS, so no lane selects
// or negates anything inside the loop.
// Each tile's accumulators start from init(p, r); out(p, r, value) receives
// each complex output entry (row p, column r).
// WS is the row stride of the operand in LDS (a wider operand's column block
// can be multiplied on its own).
template <typename T, int RG, int PF, int WS = lds_width<T>(RG), bool LATE_INIT = false, typename Init, typename Out>
__device__ __forceinline__ void plane_product(ChunkStream<T>& cs, const cpx<T>* Bs, int wave, int nwaves, int lane,
                                              cpx<T> (&a)[PF][4], Init&& init, Out&& out) {
  using V4 = typename Mfma<T>::v4;
  constexpr int W = WS;
  constexpr int NT = RG >= 16 ? RG / 16 : 1;  // 16-column MFMA tiles
  // GAUSS (one 16-column tile, accumulators from zero): the complex product
  // from three real ones, P1 = Re S Re T, P2 = Im S Im T,
  // P3 = (Re S + Im S)(Re T + Im T): Re C = P1 - P2, Im C = P3 - P1 - P2
  constexpr bool GAUSS = LATE_INIT && RG == 16;
  constexpr int NACC = GAUSS ? 3 : (RG >= 16 ? 2 : 1);
  const int lrow = lane & 15, lg = lane >> 4;
  const int nct = cs.nct, total = cs.ntw * cs.nct;
  const cpx<T>* Bcol = Bs + 4 * lg * W + lrow;
  V4 acc[NT][NACC];
  [[maybe_unused]] cpx<T> y0s[LATE_INIT ? NT : 1][4];
  int mt = wave, kc = 0;
  for (int c0 = 0; c0 < total; c0 += PF) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      if (c0 + j < total) {
        if (kc == 0) {  // accumulators start from init(p, r) (zero, or y_k in the backward sweep)
          if constexpr (RG >= 16 && LATE_INIT) {
            // FP64: the tile starts from zero and y_k is added at its output, so
            // the load of y_k is in flight during the tile's products
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
              for (int q = 0; q < NACC; ++q) acc[nt][q] = V4{0, 0, 0, 0};
#pragma unroll
              for (int v = 0; v < 4; ++v) y0s[nt][v] = init(mt * 16 + Mfma<T>::row(lg, v), nt * 16 + lrow);
            }
          } else if constexpr (RG >= 16) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const cpx<T> y0 = init(mt * 16 + Mfma<T>::row(lg, v), nt * 16 + lrow);
                acc[nt][0][v] = y0.re;
                acc[nt][1][v] = y0.im;
              }
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const cpx<T> y0 = init(mt * 16 + Mfma<T>::row(lg, v), lrow & 7);
              acc[0][0][v] = lrow < 8 ? y0.re : y0.im;
            }
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const T are = a[j][t].re, aim = a[j][t].im;
          if constexpr (GAUSS) {
            const T asum = are + aim;
            const cpx<T> tv = Bcol[(kc + t) * W];
            acc[0][0] = Mfma<T>::op(are, tv.re, acc[0][0]);
            acc[0][1] = Mfma<T>::op(aim, tv.im, acc[0][1]);
            acc[0][2] = Mfma<T>::op(asum, tv.re + tv.im, acc[0][2]);
          } else if constexpr (RG >= 16) {
            const T naim = -aim;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
              const cpx<T> tv = Bcol[(kc + t) * W + nt * 16];
              acc[nt][0] = Mfma<T>::op(are, tv.re, acc[nt][0]);
              acc[nt][1] = Mfma<T>::op(are, tv.im, acc[nt][1]);
              acc[nt][0] = Mfma<T>::op(naim, tv.im, acc[nt][0]);
              acc[nt][1] = Mfma<T>::op(aim, tv.re, acc[nt][1]);
            }
          } else {
            const cpx<T> tv = Bcol[(kc + t) * W];  // (B1, B2) of this lane
            acc[0][0] = Mfma<T>::op(are, tv.re, acc[0][0]);
            acc[0][0] = Mfma<T>::op(aim, tv.im, acc[0][0]);
          }
        }
        kc += 16;
        if (kc == 16 * nct) {
          if constexpr (GAUSS) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const T re = acc[0][0][v] - acc[0][1][v], im = (acc[0][2][v] - acc[0][0][v]) - acc[0][1][v];
              out(mt * 16 + Mfma<T>::row(lg, v), lrow, mk<T>(y0s[0][v].re + re, y0s[0][v].im + im));
            }
          } else if constexpr (RG >= 16 && LATE_INIT) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                out(mt * 16 + Mfma<T>::row(lg, v), nt * 16 + lrow,
                    mk<T>(y0s[nt][v].re + acc[nt][0][v], y0s[nt][v].im + acc[nt][1][v]));
          } else if constexpr (RG >= 16) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                out(mt * 16 + Mfma<T>::row(lg, v), nt * 16 + lrow, mk<T>(acc[nt][0][v], acc[nt][1][v]));
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const T im = __shfl_xor(acc[0][0][v], 8);  // column lrow + 8 holds Im of column lrow
              if (lrow < 8) out(mt * 16 + Mfma<T>::row(lg, v), lrow, mk<T>(acc[0][0][v], im));
            }
          }
          kc = 0;
          mt += nwaves;
        }
      }
      cs.next(a[j]);  // chunk c0 + j + PF (unconditional)
    }
  }
}

// Store entry (p, r) of the plane operand in the layout plane_product reads.
template <typename T, int RG>
__device__ __forceinline__ void put_operand(cpx<T>* Bs, int p, int r, cpx<T> v) {
  constexpr int W = lds_width<T>(RG);
  if constexpr (RG >= 16) {
    Bs[p * W + r] = v;
  } else {
    Bs[p * W + r] = mk<T>(v.re, -v.im);     // lane r:     B1 = Re T, B2 = -Im T
    Bs[p * W + r + 8] = mk<T>(v.im, v.re);  // lane r + 8: B1 = Im T, B2 = Re T
  }
}

// Planes too large for their operand in LDS: the operand of an item (the
// RG = 8 split layout, [bp][16]) lives in a slice of global memory and is read
// back through L2.  Each chunk's operand values are loaded together with its
// factor values: lane l reads rows 16 c + 4 (l/16) + t, t < 4, column l % 16 of
// the operand for chunk c, the rows its A values multiply.
template <typename T>
__device__ __forceinline__ void next_chunk_gl(ChunkStream<T>& cs, const cpx<T>* __restrict__ bcol, cpx<T> (&a)[4],
                                              cpx<T> (&b)[4]) {
  const int c = cs.tile >= cs.ntw ? cs.nct - 1 : cs.chunk;  // the chunk this load covers (clamped past the end)
  cs.next(a);
  const cpx<T>* q = bcol + (long long)c * 16 * 16;
#pragma unroll
  for (int t = 0; t < 4; ++t) b[t] = q[t * 16];
}

// plane_product for RG = 8 with the operand in global memory (bcol = operand +
// 4 (lane/16) 16 + lane % 16); a and b hold the PF chunks in flight.
template <typename T, int PF, typename Init, typename Out>
__device__ __forceinline__ void plane_product_gl(ChunkStream<T>& cs, const cpx<T>* __restrict__ bcol, int wave,
                                                 int nwaves, int lane, cpx<T> (&a)[PF][4], cpx<T> (&b)[PF][4],
                                                 Init&& init, Out&& out) {
  using V4 = typename Mfma<T>::v4;
  const int lrow = lane & 15, lg = lane >> 4;
  const int nct = cs.nct, total = cs.ntw * cs.nct;
  V4 acc;
  int mt = wave, kc = 0;
  for (int c0 = 0; c0 < total; c0 += PF) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      if (c0 + j < total) {
        if (kc == 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const cpx<T> y0 = init(mt * 16 + Mfma<T>::row(lg, v), lrow & 7);
            acc[v] = lrow < 8 ? y0.re : y0.im;
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc = Mfma<T>::op(a[j][t].re, b[j][t].re, acc);
          acc = Mfma<T>::op(a[j][t].im, b[j][t].im, acc);
        }
        kc += 16;
        if (kc == 16 * nct) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T im = __shfl_xor(acc[v], 8);  // column lrow + 8 holds Im of column lrow
            if (lrow < 8) out(mt * 16 + Mfma<T>::row(lg, v), lrow, mk<T>(acc[v], im));
          }
          kc = 0;
          mt += nwaves;
        }
      }
      next_chunk_gl(cs, bcol, a[j], b[j]);  // chunk c0 + j + PF (unconditional)
    }
  }
}

// LDS holds only the right operand T of the plane product; the plane solutions
// y_k / x_k live in yloc and reach the other waves of the workgroup through L2
// (workgroup-scope release/acquire around the barrier).
// Waves per workgroup at most: 12 in FP64 (three per SIMD leave 168 registers
// for the operand build and the product), 16 in FP32.
template <typename T>
constexpr int fused_max_waves() {
  return sizeof(T) == 8 ? 12 : 16;
}

// One (box, right-hand-side group) item of the batched local solves: plane
// vectors in yloc (plane k, row p, column r at (k*bp + p)*nrhs + r0 + r),
// plane couplings in the factor precision, and the box's place in the grid.
template <typename T, int RG>
struct BoxCtx {
  Sub sb;
  int r0, nrg, nrhs, gnx, gny;
  cpx<T>* yb;
  const cpx<T>* cbox;
  const z64* u;
  z64* z;
  const z64* add;

  __device__ __forceinline__ BoxCtx(const Sub* subs, int item, int ngroups, int nrhs_, const cpx<T>* cpl,
                                    const z64* u_, z64* z_, const z64* add_, int gnx_, int gny_, cpx<T>* yloc) {
    sb = subs[item / ngroups];
    r0 = (item % ngroups) * RG;
    nrhs = nrhs_;
    nrg = min(RG, nrhs - r0);
    gnx = gnx_;
    gny = gny_;
    yb = yloc + sb.vec_off * (long long)nrhs + r0;
    cbox = cpl + sb.node_off * 18;
    u = u_;
    z = z_;
    add = add_;
  }
  __device__ __forceinline__ long long gnode(int k, int p) const {
    const int px = p % sb.ex, py = p / sb.ex;
    return (sb.elo[0] + px) + (long long)gnx * ((sb.elo[1] + py) + (long long)gny * (sb.elo[2] + k));
  }
  // Operand build: each thread handles NE columns r, r + LP, ... of one node p
  // (LP = RG / NE lanes per node), so the nine coupling coefficients are loaded
  // once for NE entries.  All loads of an entry group are issued before any is
  // used: indices are clamped into the box (and columns into the batch) and
  // the coefficients of clamped taps are zero.  Offsets from the wave-uniform
  // bases are 32-bit (plane vectors of a box stay far below 2^31 elements).
  static constexpr int NE = sizeof(T) == 8 ? 1 : 2, LP = RG / NE;
  // v[j] = (u_k - L_k y_{k-1}) (dz = -1, with_u) or -U_k x_{k+1} (dz = +1) at (p, r + j LP)
  // Taps [I0, I0 + N) of the nine couplings: all loads of the batch are issued
  // before any is used.
  template <int I0, int N>
  __device__ __forceinline__ void taps(int p, int px, int py, int ro, int yo, const int (&col)[NE],
                                       cpx<T> (&v)[NE]) const {
    const int ex = sb.ex, ey = sb.ey;
    cpx<T> cv[N];
    cpx<T> yv[N][NE];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const int i = I0 + n;
      const int cx = px + i % 3 - 1, cy = py + i / 3 - 1;
      const bool in = cx >= 0 && cx < ex && cy >= 0 && cy < ey;  // taps leaving the box have zero coefficients
      const int q = yo + (in ? cx + ex * cy : p) * nrhs;
      cv[n] = cbox[ro + i];
#pragma unroll
      for (int j = 0; j < NE; ++j) yv[n][j] = yb[q + col[j]];
    }
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
      for (int j = 0; j < NE; ++j) cfms(v[j], cv[n], yv[n][j]);
  }
  // SPLIT: the nine taps in two batches (five, then four), which halves the
  // registers the build holds at once, for kernels sized for more waves per SIMD.
  template <bool SPLIT = false>
  __device__ __forceinline__ void build(int k, int p, int r, int dz, bool with_u, cpx<T> (&v)[NE]) const {
    const int b = sb.b, ex = sb.ex, bp = sb.bp;
#pragma unroll
    for (int j = 0; j < NE; ++j) v[j] = mk<T>(0, 0);
    if (p >= b) return;
    int col[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) col[j] = min(r + j * LP, nrg - 1);
    if (with_u) {
      const long long gu = gnode(k, p) * nrhs + r0;
#pragma unroll
      for (int j = 0; j < NE; ++j) v[j] = ccast<T>(u[gu + col[j]]);
    }
    if (k + dz < 0 || k + dz >= sb.ez) return;
    const int px = p % ex, py = p / ex;
    const int ro = (k * b + p) * 18 + (dz + 1) / 2 * 9;
    const int yo = (k + dz) * bp * nrhs;
    if constexpr (SPLIT) {
      taps<0, 5>(p, px, py, ro, yo, col, v);
      taps<5, 4>(p, px, py, ro, yo, col, v);
    } else {
      taps<0, 9>(p, px, py, ro, yo, col, v);
    }
  }
  // operand of plane k into Bs, threads t0, t0 + nt, ... of the workgroup.
  // With cmax (nt a multiple of LP, so each thread keeps its columns), the
  // largest |Re| or |Im| of every operand column is also reduced into
  // cmax[column] (float bits, atomic max; cmax zeroed by the caller).
  template <bool SPLIT = false, bool CMAX = false>
  __device__ __forceinline__ void build_plane(int k, int dz, bool with_u, cpx<T>* Bs, int t0, int nt,
                                              unsigned* cmax = nullptr) const {
    T m[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) m[j] = 0;
#pragma unroll 1
    for (int e = t0; e < sb.bp * LP; e += nt) {
      const int p = e / LP, r = e % LP;
      cpx<T> v[NE];
      build<SPLIT>(k, p, r, dz, with_u, v);
#pragma unroll
      for (int j = 0; j < NE; ++j) {
        const cpx<T> w = r + j * LP < nrg ? v[j] : mk<T>(0, 0);
        put_operand<T, RG>(Bs, p, r + j * LP, w);
        if constexpr (CMAX) m[j] = fmax(m[j], fmax(fabs(w.re), fabs(w.im)));
      }
    }
    if constexpr (CMAX) {
      static_assert(sizeof(T) == 4, "column maxima of complex FP32 operands");
      const int lane = t0 & 63, r = t0 % LP;
#pragma unroll
      for (int j = 0; j < NE; ++j) {
        for (int off = LP; off < 64; off <<= 1) m[j] = fmax(m[j], __shfl_xor(m[j], off));
        if (lane < LP) atomicMax(&cmax[r + j * LP], __float_as_uint(m[j]));
      }
    }
  }
  // The same operand with NEB columns of one node per thread (LPB = RG / NEB
  // lanes per node; NEB = 2 in FP64 and 4 in FP32, where build() takes one
  // and two): each coupling coefficient is loaded once for NEB columns, and
  // the taps go in batches of TB whose loads are all issued before any is
  // used, so the build waits on L2 fewer times per entry.  Every entry sums
  // its terms in the order build() does, so the operand is the same bit for
  // bit.
  // ys: the neighbouring plane's solution in LDS ([bp][RG], this item's columns), else read from yloc
  template <int NEB, int TB = 9, bool CMAX = false, bool YS = false>
  __device__ __forceinline__ void build_plane_ne(int k, int dz, bool with_u, cpx<T>* Bs, int t0, int nt,
                                                 unsigned* cmax = nullptr, const cpx<T>* ys = nullptr) const {
    constexpr int LPB = RG / NEB;
    T m[NEB];
#pragma unroll
    for (int j = 0; j < NEB; ++j) m[j] = 0;
    const int b = sb.b, ex = sb.ex, ey = sb.ey, bp = sb.bp;
    const bool taps_on = k + dz >= 0 && k + dz < sb.ez;
    const int yo = (k + dz) * bp * nrhs;
#pragma unroll 1
    for (int e = t0; e < bp * LPB; e += nt) {
      const int p = e / LPB, r = e % LPB;
      cpx<T> v[NEB];
#pragma unroll
      for (int j = 0; j < NEB; ++j) v[j] = mk<T>(0, 0);
      if (p < b) {
        int col[NEB];
#pragma unroll
        for (int j = 0; j < NEB; ++j) col[j] = min(r + j * LPB, nrg - 1);
        if (with_u) {
          const long long gu = gnode(k, p) * nrhs + r0;
#pragma unroll
          for (int j = 0; j < NEB; ++j) v[j] = ccast<T>(u[gu + col[j]]);
        }
        if (taps_on) {
          const int px = p % ex, py = p / ex;
          const int ro = (k * b + p) * 18 + (dz + 1) / 2 * 9;
          // the nine taps in batches of TB: all loads of a batch are issued before any is used
#pragma unroll
          for (int i0 = 0; i0 < 9; i0 += TB) {
            cpx<T> cv[TB], yv[TB][NEB];
#pragma unroll
            for (int n = 0; n < TB; ++n) {
              const int i = min(i0 + n, 8);
              const int cx = px + i % 3 - 1, cy = py + i / 3 - 1;
              const bool in = cx >= 0 && cx < ex && cy >= 0 && cy < ey;  // taps leaving the box have zero coefficients
              const int q = in ? cx + ex * cy : p;
              cv[n] = cbox[ro + i];
              if constexpr (YS) {
#pragma unroll
                for (int j = 0; j < NEB; ++j) yv[n][j] = ys[q * RG + col[j]];
              } else {
                const int qi = yo + q * nrhs;
#pragma unroll
                for (int j = 0; j < NEB; ++j) yv[n][j] = yb[qi + col[j]];
              }
            }
#pragma unroll
            for (int n = 0; n < TB; ++n)
              if (i0 + n < 9)
#pragma unroll
                for (int j = 0; j < NEB; ++j) cfms(v[j], cv[n], yv[n][j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < NEB; ++j) {
        const cpx<T> w = r + j * LPB < nrg ? v[j] : mk<T>(0, 0);
        put_operand<T, RG>(Bs, p, r + j * LPB, w);
        if constexpr (CMAX) m[j] = fmax(m[j], fmax(fabs(w.re), fabs(w.im)));
      }
    }
    if constexpr (CMAX) {  // column maxima, as build_plane's (nt a multiple of 64, so lanes keep their columns)
      static_assert(sizeof(T) == 4, "column maxima of complex FP32 operands");
      const int lane = t0 & 63, r = t0 % LPB;
#pragma unroll
      for (int j = 0; j < NEB; ++j) {
        for (int off = LPB; off < 64; off <<= 1) m[j] = fmax(m[j], __shfl_xor(m[j], off));
        if (lane < LPB) atomicMax(&cmax[r + j * LPB], __float_as_uint(m[j]));
      }
    }
  }
  template <int NEB, int TB = 9, bool CMAX = false, bool YS = false>
  __device__ __forceinline__ void build_step_ne(int s, cpx<T>* Bs, int t0, int nt, unsigned* cmax = nullptr,
                                                const cpx<T>* ys = nullptr) const {
    if (s < sb.ez) build_plane_ne<NEB, TB, CMAX, YS>(s, -1, true, Bs, t0, nt, cmax, ys);
    else build_plane_ne<NEB, TB, CMAX, YS>(plane_of(s), +1, false, Bs, t0, nt, cmax, ys);
  }
  // core node (k, p) of the box: z = x (+ add)
  __device__ __forceinline__ void scatter(int k, int p, int r, cpx<T> val) const {
    if (k < sb.lo[2] - sb.elo[2] || k >= sb.hi[2] - sb.elo[2] || p >= sb.b || r >= nrg) return;
    const int px = p % sb.ex, py = p / sb.ex;
    if (px < sb.lo[0] - sb.elo[0] || px >= sb.hi[0] - sb.elo[0] || py < sb.lo[1] - sb.elo[1] ||
        py >= sb.hi[1] - sb.elo[1])
      return;
    const long long gi = gnode(k, p) * nrhs + r0 + r;
    z64 o = ccast<double>(val);
    if (add) o += add[gi];
    z[gi] = o;
  }
  // Step s of the block-tridiagonal solve: s < ez is forward plane k = s,
  // then backward planes k = ez - 2, ..., 0.
  __device__ __forceinline__ int nsteps() const { return 2 * sb.ez - 1; }
  __device__ __forceinline__ int plane_of(int s) const { return s < sb.ez ? s : 2 * sb.ez - 2 - s; }
  template <bool SPLIT = false, bool CMAX = false>
  __device__ __forceinline__ void build_step(int s, cpx<T>* Bs, int t0, int nt, unsigned* cmax = nullptr) const {
    if (s < sb.ez) build_plane<SPLIT, CMAX>(s, -1, true, Bs, t0, nt, cmax);
    else build_plane<SPLIT, CMAX>(plane_of(s), +1, false, Bs, t0, nt, cmax);
  }
  __device__ __forceinline__ const cpx<T>* factor(const cpx<T>* sinv, int s) const {
    return sinv + sb.mat_off + (long long)plane_of(s) * sb.bp * sb.bp;
  }
  // accumulator start: zero forward, y_k backward (x_k = y_k + Sinv_k T with
  // the operand holding -U_k x_{k+1}; column clamped into the group)
  __device__ __forceinline__ cpx<T> init(int s, int p, int r) const {
    if (s < sb.ez) return mk<T>(0, 0);
    return yb[((long long)plane_of(s) * sb.bp + p) * nrhs + min(r, nrg - 1)];
  }
  // product output: forward y_k (and x = y on the last plane), backward x_k
  __device__ __forceinline__ void output(int s, int p, int r, cpx<T> val) const {
    if (r >= nrg) return;
    const int k = plane_of(s);
    yb[((long long)k * sb.bp + p) * nrhs + r] = val;
    if (s >= sb.ez - 1) scatter(k, p, r, val);
  }
};

// LDS holds only the right operand T of the plane product; the plane solutions
// y_k / x_k live in yloc and reach the other waves of the workgroup through L2
// (workgroup-scope release/acquire around the barrier).  One workgroup per
// item, all its waves building and then multiplying each plane in turn.
// MINW > 1: compiled for at least MINW waves per SIMD (two 9-wave workgroups
// on a compute unit at MINW = 5), with the operand build's taps split in two.
// PAIR: the workgroup takes two right-hand-side groups of one box (items
// 2j, 2j + 1 of the box), each on half of its waves with its own operand slot
// (half_elems elements apart in LDS).  Both halves stream the same factor
// chunks within the same plane step, so the second read of each chunk mostly
// hits L2, and the factors cross HBM about once per application.
// YLDS (groups of 16): each item also keeps its last plane solution in LDS
// ([bp][RG] at ys_off elements after its operand), written by the products
// beside yloc; the next plane's operand build reads its neighbours there, so a
// plane step needs only a workgroup barrier, and the release/acquire through
// L2 happens once, when the forward sweep turns (the backward products start
// from y_k in yloc).
template <typename T, int RG, int PF, int MINW, bool PAIR, bool YLDS = false>
__global__ void __launch_bounds__(64 * fused_max_waves<T>(), MINW) k_oras_fused(const Sub* __restrict__ subs, int ngroups, int nrhs,
                                                   const cpx<T>* __restrict__ cpl, const cpx<T>* __restrict__ sinv,
                                                   const z64* __restrict__ u, z64* __restrict__ z,
                                                   const z64* __restrict__ add, int gnx, int gny,
                                                   cpx<T>* __restrict__ yloc, int half_elems, int ys_off) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int FT = blockDim.x, nwaves = FT >> 6;
  // the item's waves (wave-uniform values, kept in scalar registers)
  int hw = nwaves, half = 0, wv = __builtin_amdgcn_readfirstlane(wave), ht = tid;
  if constexpr (PAIR) {
    hw = nwaves >> 1;
    half = __builtin_amdgcn_readfirstlane(wave >= hw ? 1 : 0);
    wv = __builtin_amdgcn_readfirstlane(wave - half * hw);
    ht = tid - half * hw * 64;
  }
  cpx<T>* Bs = reinterpret_cast<cpx<T>*>(smem_raw) + half * half_elems;
  // items of one box (its RHS groups) and neighbouring boxes go to the same XCD
  // back to back, so the groups' reads of the box's factors meet in its L2
  const int wg = (int)xcd_contiguous(blockIdx.x, gridDim.x);
  const int item = PAIR ? (wg / (ngroups / 2)) * ngroups + 2 * (wg % (ngroups / 2)) + half : wg;
  const BoxCtx<T, RG> bx(subs, item, ngroups, nrhs, cpl, u, z, add, gnx, gny, yloc);
  const int bp = bx.sb.bp, ns = bx.nsteps();
  for (int st = 0; st < ns; ++st) {
    cpx<T> a[PF][4];
    ChunkStream<T> cs;
    if constexpr (sizeof(T) == 8 && MINW == 1 && RG >= 16) {
      // the first factor chunk is in flight during the operand build
      cs = ChunkStream<T>(bx.factor(sinv, st), bp, wv, hw, lane);
      cs.next(a[0]);
      bx.template build_step_ne<2, 9, false, YLDS>(st, Bs, ht, hw * 64, nullptr, Bs + ys_off);
#pragma unroll
      for (int j = 1; j < PF; ++j) cs.next(a[j]);
    } else if constexpr (sizeof(T) == 4 && RG >= 16) {
      bx.template build_step_ne<4, 5, false, YLDS>(st, Bs, ht, hw * 64, nullptr, Bs + ys_off);
      cs = prefetch_tile<T, PF>(bx.factor(sinv, st), bp, wv, hw, lane, a);  // across the barrier
    } else {
      bx.template build_step<(MINW > 1)>(st, Bs, ht, hw * 64);
      cs = prefetch_tile<T, PF>(bx.factor(sinv, st), bp, wv, hw, lane, a);  // across the barrier
    }
    __syncthreads();
    constexpr bool late = (sizeof(T) == 8 && MINW == 1 && RG >= 16) || (sizeof(T) == 4 && RG >= 16 && !PAIR);
    plane_product<T, RG, PF, lds_width<T>(RG), late>(
        cs, Bs, wv, hw, lane, a, [&](int p, int r) { return bx.init(st, p, r); },
        [&](int p, int r, cpx<T> val) {
          bx.output(st, p, r, val);
          if constexpr (YLDS) Bs[ys_off + p * RG + r] = val;
        });
    if constexpr (YLDS) {
      if (st == bx.sb.ez - 1) wg_sync_global();  // the forward solutions in yloc, for the backward products
      else __syncthreads();
    } else {
      wg_sync_global();
    }
  }
}

// The same sweep for planes whose operand does not fit in LDS: the operand of
// item i is tglob[i][bpmax][16] (RG = 8 split layout) in global memory, built
// by all waves, published by the workgroup-scope release/acquire barrier, and
// streamed back through L2 with the factor chunks.
template <typename T, int PF>
__global__ void __launch_bounds__(64 * fused_max_waves<T>()) k_oras_gl(const Sub* __restrict__ subs, int ngroups, int nrhs,
                                                   const cpx<T>* __restrict__ cpl, const cpx<T>* __restrict__ sinv,
                                                   const z64* __restrict__ u, z64* __restrict__ z,
                                                   const z64* __restrict__ add, int gnx, int gny,
                                                   cpx<T>* __restrict__ yloc, cpx<T>* __restrict__ tglob, int bpmax) {
  const int item = (int)xcd_contiguous(blockIdx.x, gridDim.x);
  const BoxCtx<T, 8> bx(subs, item, ngroups, nrhs, cpl, u, z, add, gnx, gny, yloc);
  cpx<T>* Bs = tglob + (long long)item * bpmax * 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int FT = blockDim.x, nwaves = FT >> 6;
  const int bp = bx.sb.bp, ns = bx.nsteps();
  const cpx<T>* bcol = Bs + 4 * (lane >> 4) * 16 + (lane & 15);
  for (int st = 0; st < ns; ++st) {
    bx.build_step(st, Bs, tid, FT);
    wg_sync_global();  // the operand, written by every wave, is read by every wave
    cpx<T> a[PF][4], b[PF][4];
    ChunkStream<T> cs(bx.factor(sinv, st), bp, wave, nwaves, lane);
#pragma unroll
    for (int j = 0; j < PF; ++j) next_chunk_gl(cs, bcol, a[j], b[j]);
    plane_product_gl<T, PF>(
        cs, bcol, wave, nwaves, lane, a, b, [&](int p, int r) { return bx.init(st, p, r); },
        [&](int p, int r, cpx<T> val) { bx.output(st, p, r, val); });
    wg_sync_global();
  }
}

// ---- approximate local solves: plane inverses in complex FP16 ----------------
//
// Factor storage of the approximate form: plane k of a box holds Sinv_k 2^-e
// (e = sexp[id maxez + k], id = the box's Sub::id, chosen so that the largest
// |Re| or |Im| lies in [2^13, 2^14)), in blocks of 16 bytes: for row p and column group g
// (columns 4g .. 4g + 3) the four real parts, then the four imaginary parts, as
// FP16.  The operand T stays complex FP32 in LDS; each column is scaled by a
// power of two (its largest |Re| or |Im| to [2^13, 2^14)) and rounded to FP16
// as the product reads it.  Products on v_mfma_f32_16x16x16_f16, FP32
// accumulation; the accumulators start from y_k and end as the output scaled
// by the inverse powers of two (exact).
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
union H4U {
  uint2 u;
  h4 h;
};

// A wave's 16-row tiles of a FP16 plane inverse, 16 columns (one 16-byte block
// per lane: row wave 16 + lane % 16, column group 4 c + lane / 16) per chunk,
// unconditional loads clamped past the end as in ChunkStream.
struct HalfStream {
  const uint4* base;
  long long tile_step;
  int nct, ntw, tile, chunk;
  __device__ __forceinline__ HalfStream(const uint4* Sk, int bp, int wave, int nwaves, int lane) {
    const int nmt = bp >> 4, bq = bp >> 2;
    nct = nmt;
    ntw = wave < nmt ? (nmt - wave + nwaves - 1) / nwaves : 0;
    base = Sk + (long long)(min(wave, nmt - 1) * 16 + (lane & 15)) * bq + (lane >> 4);
    tile_step = (long long)nwaves * 16 * bq;
    tile = 0;
    chunk = 0;
  }
  __device__ __forceinline__ uint4 next() {
    const bool past = tile >= ntw;
    const uint4* p = base + (past ? (long long)(ntw > 0 ? ntw - 1 : 0) * tile_step + 4 * (nct - 1)
                                  : (long long)tile * tile_step + 4 * chunk);
    const uint4 v = *p;
    if (++chunk == nct) {
      chunk = 0;
      ++tile;
    }
    return v;
  }
};

// Power-of-two exponent that maps m (>= 0) into [2^13, 2^14): m = f 2^x, f in [0.5, 1).
__device__ __forceinline__ int half_shift(float m) {
  int x = 0;
  (void)frexpf(m, &x);
  return m > 0.f ? x - 14 : 0;
}

// Sinv_k T for the wave's tiles with the FP16 factors; cmax holds the operand's
// column maxima (float bits), sS the plane's scale exponent.
template <int RG, int PF, typename Init, typename Out>
__device__ __forceinline__ void plane_product_half(HalfStream& cs, const c32* __restrict__ Bs,
                                                   const unsigned* cmax, int sS, int wave, int nwaves, int lane,
                                                   uint4 (&a)[PF], Init&& init, Out&& out) {
  constexpr int W = lds_width<float>(RG), NT = RG / 16;
  const int lrow = lane & 15, lg = lane >> 4;
  int sT[NT];
  float tin[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    sT[nt] = half_shift(__uint_as_float(cmax[nt * 16 + lrow]));
    tin[nt] = ldexpf(1.f, -sT[nt]);
  }
  const c32* Bcol = Bs + 4 * lg * W + lrow;
  const int nct = cs.nct, total = cs.ntw * cs.nct;
  f4v acc[NT][2];
  int mt = wave, kc = 0;
  for (int c0 = 0; c0 < total; c0 += PF) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      if (c0 + j < total) {
        if (kc == 0) {  // start from y_k (backward) or zero, in the product's scale
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const float f = ldexpf(1.f, -(sS + sT[nt]));
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const c32 y0 = init(mt * 16 + Mfma<float>::row(lg, v), nt * 16 + lrow);
              acc[nt][0][v] = y0.re * f;
              acc[nt][1][v] = y0.im * f;
            }
          }
        }
        H4U sr, si;
        sr.u = make_uint2(a[j].x, a[j].y);
        si.u = make_uint2(a[j].z, a[j].w);
        const h4 nsi = -si.h;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          h4 tre, tim;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const c32 tv = Bcol[(kc + t) * W + nt * 16];
            tre[t] = (_Float16)(tv.re * tin[nt]);
            tim[t] = (_Float16)(tv.im * tin[nt]);
          }
          acc[nt][0] = __builtin_amdgcn_mfma_f32_16x16x16f16(sr.h, tre, acc[nt][0], 0, 0, 0);
          acc[nt][0] = __builtin_amdgcn_mfma_f32_16x16x16f16(nsi, tim, acc[nt][0], 0, 0, 0);
          acc[nt][1] = __builtin_amdgcn_mfma_f32_16x16x16f16(sr.h, tim, acc[nt][1], 0, 0, 0);
          acc[nt][1] = __builtin_amdgcn_mfma_f32_16x16x16f16(si.h, tre, acc[nt][1], 0, 0, 0);
        }
        kc += 16;
        if (kc == 16 * nct) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const float f = ldexpf(1.f, sS + sT[nt]);
#pragma unroll
            for (int v = 0; v < 4; ++v)
              out(mt * 16 + Mfma<float>::row(lg, v), nt * 16 + lrow, mk<float>(acc[nt][0][v] * f, acc[nt][1][v] * f));
          }
          kc = 0;
          mt += nwaves;
        }
      }
      a[j] = cs.next();  // chunk c0 + j + PF (unconditional)
    }
  }
}

// The one-workgroup-per-item sweep with FP16 factors: build (complex FP32
// operand in LDS, column maxima into cmax), barrier, product, barrier.  The
// column maxima alternate between two buffers; the one not in use is cleared
// during the build.  YLDS: the plane solutions are also kept in LDS
// ([bp][RG] at ys_off elements), as in k_oras_fused.
template <int RG, int PF, bool YLDS = false>
__global__ void __launch_bounds__(64 * 16) k_oras_half(const Sub* __restrict__ subs, int ngroups, int nrhs,
                                                       const c32* __restrict__ cpl, const uint4* __restrict__ sinv16,
                                                       const int* __restrict__ sexp, int maxez,
                                                       const z64* __restrict__ u, z64* __restrict__ z,
                                                       const z64* __restrict__ add, int gnx, int gny,
                                                       c32* __restrict__ yloc, int ys_off) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  c32* Bs = reinterpret_cast<c32*>(smem_raw);
  __shared__ unsigned cmax[2][RG];
  const int item = (int)xcd_contiguous(blockIdx.x, gridDim.x);
  const BoxCtx<float, RG> bx(subs, item, ngroups, nrhs, cpl, u, z, add, gnx, gny, yloc);
  const int box = bx.sb.id;  // the exponents are stored in box order
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int FT = blockDim.x, nwaves = FT >> 6;
  const int bp = bx.sb.bp, ns = bx.nsteps();
  for (int i = tid; i < 2 * RG; i += FT) (&cmax[0][0])[i] = 0u;
  __syncthreads();
  for (int st = 0; st < ns; ++st) {
    const int cb = st & 1, k = bx.plane_of(st);
    for (int i = tid; i < RG; i += FT) cmax[cb ^ 1][i] = 0u;
    bx.template build_step_ne<4, 5, true, YLDS>(st, Bs, tid, FT, cmax[cb], Bs + ys_off);
    uint4 a[PF];
    HalfStream cs(sinv16 + (bx.sb.mat_off + (long long)k * bp * bp) / 4, bp, wave, nwaves, lane);
#pragma unroll
    for (int j = 0; j < PF; ++j) a[j] = cs.next();
    __syncthreads();
    plane_product_half<RG, PF>(
        cs, Bs, cmax[cb], sexp[box * maxez + k], wave, nwaves, lane, a,
        [&](int p, int r) { return bx.init(st, p, r); },
        [&](int p, int r, c32 val) {
          bx.output(st, p, r, val);
          if constexpr (YLDS) Bs[ys_off + p * RG + r] = val;
        });
    if constexpr (YLDS) {
      if (st == bx.sb.ez - 1) wg_sync_global();  // the forward solutions in yloc, for the backward products
      else __syncthreads();
    } else {
      wg_sync_global();
    }
  }
}

// Plane inverses of one level to the FP16 storage above: one workgroup per
// (plane, box); the plane's largest |Re| or |Im| sets its exponent.
__global__ void __launch_bounds__(256) k_to_half(const Sub* __restrict__ subs, int maxez, const c32* __restrict__ sinv,
                                                 uint4* __restrict__ sinv16, int* __restrict__ sexp) {
  const int k = blockIdx.x, s = blockIdx.y;
  const Sub sb = subs[s];
  if (k >= sb.ez) return;
  const int bp = sb.bp, bq = bp / 4;
  const long long off = sb.mat_off + (long long)k * bp * bp;
  const c32* S = sinv + off;
  float m = 0.f;
  for (long long i = threadIdx.x; i < (long long)bp * bp; i += blockDim.x)
    m = fmaxf(m, fmaxf(fabsf(S[i].re), fabsf(S[i].im)));
  __shared__ float red[4];
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const int e = half_shift(m);
  const float f = ldexpf(1.f, -e);
  if (threadIdx.x == 0) sexp[sb.id * maxez + k] = e;
  uint4* D = sinv16 + off / 4;
  for (long long i = threadIdx.x; i < (long long)bp * bq; i += blockDim.x) {
    const long long p = i / bq, g = i % bq;
    const c32* q = S + p * bp + 4 * g;
    H4U re, im;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      re.h[t] = (_Float16)(q[t].re * f);
      im.h[t] = (_Float16)(q[t].im * f);
    }
    D[i] = make_uint4(re.u.x, re.u.y, im.u.x, im.u.y);
  }
}

// Persistent pipelined variant: one workgroup per compute unit works through
// the items blockIdx.x, blockIdx.x + gridDim.x, ... with two items in flight
// (two operand slots in LDS).  In every phase the eight consumer waves (two per
// SIMD) form the plane product of one item while the producer waves build the
// next plane operand of the other, so the latency-bound build hides behind the
// matrix-core work; a barrier ends each phase.  Consumer wave cw owns the
// 16-column half nh = cw % NH (NH = RG / 16) of the tiles mt = cw / NH,
// cw / NH + 8 / NH, ..., which spreads the 16 x 16 output blocks evenly over
// the SIMDs.
constexpr int PIPE_CONSUMERS = 8;

// NW = 12 (four producer waves) or 16 (eight producer waves, for planes whose
// operand build is slower than the product with four).
template <typename T, int RG, int PF, int NW>
__global__ void __launch_bounds__(64 * NW) k_oras_pipe(const Sub* __restrict__ subs, int nitems, int ngroups,
                                                       int nrhs, int bpmax, const cpx<T>* __restrict__ cpl,
                                                       const cpx<T>* __restrict__ sinv, const z64* __restrict__ u,
                                                       z64* __restrict__ z, const z64* __restrict__ add, int gnx,
                                                       int gny, cpx<T>* __restrict__ yloc) {
  static_assert(RG >= 16, "the pipelined sweep uses the planar operand layout");
  constexpr int NH = RG / 16, W = lds_width<T>(RG);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* slots[2] = {reinterpret_cast<cpx<T>*>(smem_raw), reinterpret_cast<cpx<T>*>(smem_raw) + (long long)bpmax * W};
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool consumer = wave < PIPE_CONSUMERS;
  const int ptid = tid - 64 * PIPE_CONSUMERS, pthreads = blockDim.x - 64 * PIPE_CONSUMERS;
  const int cw = wave, nh = cw % NH;
  int item[2] = {-1, -1}, step[2] = {0, 0};
  int next = blockIdx.x;
  cpx<T> a[PF][4];
  ChunkStream<T> cs;
  for (int ph = 0;; ++ph) {
    const int B = ph & 1, P = B ^ 1;
    if (item[B] < 0 && next < nitems) {
      item[B] = next;
      step[B] = 0;
      next += gridDim.x;
    }
    if (item[B] < 0 && item[P] < 0) break;  // uniform: every thread tracks the same state
    if (consumer) {
      if (item[P] >= 0) {
        const BoxCtx<T, RG> bx(subs, item[P], ngroups, nrhs, cpl, u, z, add, gnx, gny, yloc);
        const int st = step[P];
        const cpx<T>* Bcol = slots[P] + nh * 16;
        plane_product<T, 16, PF, W>(
            cs, Bcol, cw / NH, PIPE_CONSUMERS / NH, lane, a, [&](int p, int r) { return bx.init(st, p, nh * 16 + r); },
            [&](int p, int r, cpx<T> val) { bx.output(st, p, nh * 16 + r, val); });
      }
      if (item[B] >= 0) {  // the next product: slot B's plane being built now
        const BoxCtx<T, RG> bx(subs, item[B], ngroups, nrhs, cpl, u, z, add, gnx, gny, yloc);
        cs = prefetch_tile<T, PF>(bx.factor(sinv, step[B]), bx.sb.bp, cw / NH, PIPE_CONSUMERS / NH, lane, a);
      }
    } else if (item[B] >= 0) {
      const BoxCtx<T, RG> bx(subs, item[B], ngroups, nrhs, cpl, u, z, add, gnx, gny, yloc);
      bx.build_step(step[B], slots[B], ptid, pthreads);
    }
    wg_sync_global();
    if (item[P] >= 0) {
      const int ns = 2 * subs[item[P] / ngroups].ez - 1;
      if (++step[P] == ns) item[P] = -1;
    }
  }
}

// Rounds of 16-row tiles per wave: at least enough for the wave limit; more
// rounds mean fewer waves per workgroup, so that two workgroups (two boxes) can
// share a compute unit and overlap one's operand build with the other's product.
template <typename T>
int min_rounds(int bpmax) {
  constexpr int MW = fused_max_waves<T>();
  return (bpmax / 16 + MW - 1) / MW;
}
// the paired sweep: both halves within the wave limit
template <typename T>
int pair_min_rounds(int bpmax) {
  constexpr int MW = fused_max_waves<T>() / 2;
  return (bpmax / 16 + MW - 1) / MW;
}

template <typename T>
void launch_gl_t(const Sub* subs, int nsub, int ngroups, int nrhs, int bpmax, int rounds, const cpx<T>* cpl,
                 const cpx<T>* sinv, const z64* u, z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc,
                 cpx<T>* tglob, hipStream_t s) {
  constexpr int PF = 2;
  const int nmt = bpmax / 16;
  rounds = std::max(rounds, min_rounds<T>(bpmax));
  const int nwaves = (nmt + rounds - 1) / rounds;
  hipLaunchKernelGGL((k_oras_gl<T, PF>), dim3(nsub * ngroups), dim3(64 * nwaves), 0, s, subs, ngroups, nrhs, cpl, sinv,
                     u, z, add, gnx, gny, yloc, tglob, bpmax);
}

template <typename T, int RG, int PF, int MINW, bool PAIR = false, bool YLDS = false>
void launch_fused_k(const Sub* subs, int nsub, int ngroups, int nrhs, int bpmax, int rounds, const cpx<T>* cpl,
                    const cpx<T>* sinv, const z64* u, z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc,
                    hipStream_t s) {
  const int ys_off = YLDS ? bpmax * lds_width<T>(RG) : 0;
  const int half_elems = bpmax * lds_width<T>(RG) + (YLDS ? bpmax * RG : 0);
  const size_t lds = (size_t)(PAIR ? 2 : 1) * half_elems * sizeof(cpx<T>);
  static bool attr = false;  // one per kernel instance
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_oras_fused<T, RG, PF, MINW, PAIR, YLDS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  // waves per item: the tiles spread evenly over the given number of rounds
  const int nmt = bpmax / 16;
  rounds = std::max(rounds, PAIR ? pair_min_rounds<T>(bpmax) : min_rounds<T>(bpmax));
  const int nwaves = (nmt + rounds - 1) / rounds;
  hipLaunchKernelGGL((k_oras_fused<T, RG, PF, MINW, PAIR, YLDS>), dim3(nsub * (PAIR ? ngroups / 2 : ngroups)),
                     dim3(64 * nwaves * (PAIR ? 2 : 1)), lds, s, subs, ngroups, nrhs, cpl, sinv, u, z, add, gnx, gny,
                     yloc, half_elems, ys_off);
}

// Whether the paired sweep (two groups of a box per workgroup) exists for this
// shape: an even number of groups, two operands in one CU's LDS.
template <typename T>
bool pair_fits(int rg, int bpmax, int nrhs) {
  const int ngroups = (nrhs + rg - 1) / rg;
  return rg >= 16 && ngroups % 2 == 0 && 2 * (size_t)bpmax * lds_width<T>(rg) * sizeof(cpx<T>) <= 160 * 1024;
}
// ... and its form with the plane solutions in LDS (FP64 groups of 16)
template <typename T>
bool pair_ylds_fits(int rg, int bpmax, int nrhs) {
  return sizeof(T) == 8 && rg == 16 && pair_fits<T>(rg, bpmax, nrhs) &&
         2 * (size_t)bpmax * (lds_width<T>(rg) + rg) * sizeof(cpx<T>) <= 160 * 1024;
}
// the one-group sweep with the plane solutions in LDS (groups of 16)
template <typename T>
bool item_ylds_fits(int rg, int bpmax) {
  return rg == 16 && (size_t)bpmax * (lds_width<T>(rg) + rg) * sizeof(cpx<T>) <= 160 * 1024;
}

// Whether the two-workgroups-per-CU build of the sweep exists for this shape:
// FP64 groups of 32 right-hand sides, two operands in one CU's LDS.
template <typename T>
bool lowreg_fits(int rg, int bpmax) {
  return sizeof(T) == 8 && rg == 32 && 2 * (size_t)bpmax * lds_width<T>(rg) * sizeof(cpx<T>) <= 160 * 1024;
}

template <typename T, int RG>
void launch_fused_t(const Sub* subs, int nsub, int ngroups, int nrhs, int bpmax, int rounds, bool lowreg, int pair,
                    const cpx<T>* cpl, const cpx<T>* sinv, const z64* u, z64* z, const z64* add, int gnx, int gny,
                    cpx<T>* yloc, hipStream_t s) {
  constexpr int PF = sizeof(T) == 4 ? 4 : 2;
  if constexpr (RG == 16) {
    if (pair & 2) {  // plane solutions in LDS (pair & 1: paired, complex FP64 only)
      if constexpr (sizeof(T) == 8) {
        if (pair & 1) {
          launch_fused_k<T, RG, PF, 1, true, true>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx,
                                                   gny, yloc, s);
          return;
        }
      }
      launch_fused_k<T, RG, PF, 1, false, true>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx,
                                                gny, yloc, s);
      return;
    }
  }
  if constexpr (RG >= 16) {
    if (pair & 1) {
      launch_fused_k<T, RG, PF, 1, true>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx, gny,
                                         yloc, s);
      return;
    }
  }
  if constexpr (sizeof(T) == 8 && RG == 32) {
    if (lowreg) {  // one factor chunk in flight per wave: five waves per SIMD hide the latency instead
      launch_fused_k<T, RG, 1, 5>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx, gny, yloc, s);
      return;
    }
  }
  launch_fused_k<T, RG, PF, 1>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx, gny, yloc, s);
}

// Two operand slots of the pipelined sweep must fit one compute unit's LDS.
template <typename T>
bool pipe_fits(int rg, int bpmax) {
  return rg >= 16 && 2 * (size_t)bpmax * lds_width<T>(rg) * sizeof(cpx<T>) <= 160 * 1024;
}

int compute_units() {
  static int per_device[64] = {0};
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  if (per_device[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    per_device[dev] = n;
  }
  return per_device[dev];
}

template <typename T, int RG, int NW>
void launch_pipe_t(const Sub* subs, int nsub, int ngroups, int nrhs, int bpmax, const cpx<T>* cpl, const cpx<T>* sinv,
                   const z64* u, z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc, hipStream_t s) {
  constexpr int PF = sizeof(T) == 4 ? 4 : (NW == 16 ? 1 : 2);
  const size_t lds = 2 * (size_t)bpmax * lds_width<T>(RG) * sizeof(cpx<T>);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_oras_pipe<T, RG, PF, NW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr = true;
  }
  const int nitems = nsub * ngroups;
  const int grid = std::min(nitems, compute_units());
  hipLaunchKernelGGL((k_oras_pipe<T, RG, PF, NW>), dim3(grid), dim3(64 * NW), lds, s, subs, nitems, ngroups, nrhs, bpmax,
                     cpl, sinv, u, z, add, gnx, gny, yloc);
}

}  // namespace

// LDS budget of the fused kernel (one plane operand)
constexpr size_t FUSED_LDS = 150 * 1024;

template <typename T>
bool lds_fits(int rg, int bpmax) {
  return (size_t)bpmax * lds_width<T>(rg) * sizeof(cpx<T>) <= FUSED_LDS;
}

// Widest right-hand-side group for this plane size and batch; 8 also where
// not even its operand fits in LDS (then the global-operand sweep k_oras_gl).
template <typename T>
int fused_group(int bpmax, int nrhs) {
  int rg = nrhs <= 8 ? 8 : (nrhs <= 16 ? 16 : 32);
  while (rg > 8 && !lds_fits<T>(rg, bpmax)) rg /= 2;
  return rg;
}

namespace {

template <typename T>
void launch_rg(int rg, int rounds, bool lowreg, int pair, const Sub* subs, int nsub, int nrhs, int bpmax,
               const cpx<T>* cpl, const cpx<T>* sinv, const z64* u, z64* z, const z64* add, int gnx, int gny,
               cpx<T>* yloc, cpx<T>* tglob, hipStream_t s) {
  const int ngroups = (nrhs + rg - 1) / rg;
  if (!lds_fits<T>(rg, bpmax)) {  // operand in global memory: the RG = 8 sweep k_oras_gl
    launch_gl_t<T>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx, gny, yloc, tglob, s);
    return;
  }
  if (rounds == 0) {  // pipelined persistent sweep (lowreg: the 16-wave build)
    if (rg == 16) {
      if (lowreg) launch_pipe_t<T, 16, 16>(subs, nsub, ngroups, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc, s);
      else launch_pipe_t<T, 16, 12>(subs, nsub, ngroups, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc, s);
    } else {
      if (lowreg) launch_pipe_t<T, 32, 16>(subs, nsub, ngroups, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc, s);
      else launch_pipe_t<T, 32, 12>(subs, nsub, ngroups, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc, s);
    }
    return;
  }
  switch (rg) {
    case 8:
      launch_fused_t<T, 8>(subs, nsub, ngroups, nrhs, bpmax, rounds, lowreg, pair, cpl, sinv, u, z, add, gnx, gny, yloc,
                            s);
      break;
    case 16:
      launch_fused_t<T, 16>(subs, nsub, ngroups, nrhs, bpmax, rounds, lowreg, pair, cpl, sinv, u, z, add, gnx, gny, yloc,
                            s);
      break;
    default:
      launch_fused_t<T, 32>(subs, nsub, ngroups, nrhs, bpmax, rounds, lowreg, pair, cpl, sinv, u, z, add, gnx, gny, yloc,
                            s);
      break;
  }
}

// Autotuned launch shape of the fused sweep (right-hand-side group, tile
// rounds per wave), per problem shape.
struct TuneKey {
  int es, bpmax, nsub, nrhs, gnx, gny, policy;
  bool operator<(const TuneKey& o) const {
    return std::tie(es, bpmax, nsub, nrhs, gnx, gny, policy) <
           std::tie(o.es, o.bpmax, o.nsub, o.nrhs, o.gnx, o.gny, o.policy);
  }
};
std::atomic<int> g_sweep_policy{0};
struct TuneVal {
  int rg, rounds;
  bool lowreg;  // the build for two workgroups per compute unit (lowreg_fits)
  int pair;     // bit 0: two groups of a box per workgroup (pair_fits); bit 1: plane solutions in LDS
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

// Tuning decisions persisted across processes: with HELM_TUNE_FILE set, the
// tuned launches recorded there are taken as tuned (read once, on the first
// lookup) and every new decision is appended, one line per key:
//   sweep es bpmax nsub nrhs gnx gny policy  rg rounds lowreg pair
// so that separate runs (e.g. one per hardware counter) launch the same kernels.
const char* tune_file() {
  static const char* f = std::getenv("HELM_TUNE_FILE");
  return f && *f ? f : nullptr;
}
// Whether a sweep shape (from the tuner or a tuning file) can run on this
// problem: a group the operand width allows, and the LDS its variant needs.
template <typename T>
bool admissible(const TuneVal& v, int rgmax, int bpmax, int nrhs) {
  if ((v.rg != 8 && v.rg != 16 && v.rg != 32) || v.rg > rgmax || v.rounds < 0 || v.pair < 0 || v.pair > 3) return false;
  if (!lds_fits<T>(v.rg, bpmax)) return v.pair == 0;  // the global-operand sweep
  if (v.rounds == 0) return v.pair == 0 && pipe_fits<T>(v.rg, bpmax);
  if ((v.pair & 1) && !pair_fits<T>(v.rg, bpmax, nrhs)) return false;
  if (v.pair == 3 && !pair_ylds_fits<T>(v.rg, bpmax, nrhs)) return false;
  if (v.pair == 2 && !item_ylds_fits<T>(v.rg, bpmax)) return false;
  return !v.lowreg || v.pair != 0 || lowreg_fits<T>(v.rg, bpmax);
}

void load_tune_file_locked() {  // with g_tune_mu held
  static bool loaded = false;
  if (loaded || !tune_file()) return;
  loaded = true;
  FILE* fp = std::fopen(tune_file(), "r");
  if (!fp) return;
  char tag[16];
  TuneKey k{};
  int rg, rounds, lowreg, pair;
  while (std::fscanf(fp, "%15s %d %d %d %d %d %d %d %d %d %d %d", tag, &k.es, &k.bpmax, &k.nsub, &k.nrhs, &k.gnx,
                     &k.gny, &k.policy, &rg, &rounds, &lowreg, &pair) == 12) {
    if (std::string(tag) == "sweep" && rg > 0) g_tune[k] = TuneVal{rg, rounds, lowreg != 0, pair};
  }
  std::fclose(fp);
}
void store_tune_locked(const TuneKey& k, const TuneVal& v) {  // with g_tune_mu held
  g_tune[k] = v;
  if (!tune_file()) return;
  if (FILE* fp = std::fopen(tune_file(), "a")) {
    std::fprintf(fp, "sweep %d %d %d %d %d %d %d %d %d %d %d\n", k.es, k.bpmax, k.nsub, k.nrhs, k.gnx, k.gny, k.policy,
                 v.rg, v.rounds, v.lowreg ? 1 : 0, v.pair);
    std::fclose(fp);
  }
}

}  // namespace

void set_sweep_policy(int policy) { g_sweep_policy.store(policy); }
int sweep_policy() { return g_sweep_policy.load(); }

int tuned_group(int es, int bpmax, int nsub, int nrhs, int gnx, int gny) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tune.find({es, bpmax, nsub, nrhs, gnx, gny, g_sweep_policy.load()});
  return it == g_tune.end() ? 0 : it->second.rg;
}

bool tuned_config(int es, int bpmax, int nsub, int nrhs, int gnx, int gny, int out[4]) {
  TuneVal tv{0, 0, false, 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune.find({es, bpmax, nsub, nrhs, gnx, gny, g_sweep_policy.load()});
    if (it == g_tune.end()) return false;
    tv = it->second;
  }
  const int nmt = bpmax / 16;
  const int per_item = tv.rounds == 0 ? 0 : (nmt + tv.rounds - 1) / tv.rounds;
  out[0] = tv.rg;
  out[1] = per_item;
  // the variant, numbered as the sweep policies that force it
  out[2] = tv.rounds == 0 ? (tv.lowreg ? 4 : 2) : ((tv.pair & 2) ? 6 : (tv.pair ? 5 : (tv.lowreg ? 3 : 1)));
  out[3] = tv.rounds == 0 ? (tv.lowreg ? 16 : 12) : ((tv.pair & 1) ? 2 * per_item : per_item);
  return true;
}

template <typename T>
bool oras_fused(const Sub* subs, int nsub, int bpmax, const cpx<T>* cpl, const cpx<T>* sinv, int nrhs, const z64* u,
                z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc, cpx<T>* tbuf, hipStream_t s, bool may_tune) {
  const int rgmax = fused_group<T>(bpmax, nrhs);
  if (!lds_fits<T>(rgmax, bpmax) && !tbuf) return false;  // the global-operand sweep needs its operand slices
  const int policy = g_sweep_policy.load();
  if (policy == 3 && lowreg_fits<T>(rgmax, bpmax)) {  // forced: the two-workgroups-per-CU build
    launch_rg<T>(rgmax, min_rounds<T>(bpmax), true, false, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc,
                 tbuf, s);
    return true;
  }
  if (policy == 6) {  // forced: plane solutions in LDS, paired where the groups pair
    if (pair_ylds_fits<T>(16, bpmax, nrhs)) {
      launch_rg<T>(16, pair_min_rounds<T>(bpmax), false, 3, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny,
                   yloc, tbuf, s);
      return true;
    }
    if (rgmax >= 16 && item_ylds_fits<T>(16, bpmax)) {
      launch_rg<T>(16, min_rounds<T>(bpmax), false, 2, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc,
                   tbuf, s);
      return true;
    }
  }
  if (policy == 5) {  // forced: the paired sweep with the widest group that pairs
    for (int cand = rgmax; cand >= 16; cand /= 2)
      if (pair_fits<T>(cand, bpmax, nrhs)) {
        launch_rg<T>(cand, pair_min_rounds<T>(bpmax), false, 1, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx,
                     gny, yloc, tbuf, s);
        return true;
      }
  }
  if (policy == 4) {  // forced: the 16-wave pipelined sweep with the widest group that fits
    for (int cand = rgmax; cand >= 16; cand /= 2)
      if (pipe_fits<T>(cand, bpmax)) {
        launch_rg<T>(cand, 0, true, false, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc, tbuf, s);
        return true;
      }
  }
  const TuneKey key{(int)sizeof(T), bpmax, nsub, nrhs, gnx, gny, policy};
  // policy 1: one-item sweeps only; 2: the pipelined sweep wherever it fits
  bool any_pipe = false;
  for (int cand = 8; cand <= rgmax; cand *= 2) any_pipe = any_pipe || pipe_fits<T>(cand, bpmax);
  const bool allow_pipe = policy != 1 && policy != 3, allow_item = (policy != 2 && policy != 4) || !any_pipe;
  TuneVal tv{0, 0, false, 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) tv = it->second;
  }
  if (tv.rg != 0 && !admissible<T>(tv, rgmax, bpmax, nrhs)) tv = TuneVal{0, 0, false, 0};  // a stale or foreign entry
  static const bool no_tune = std::getenv("HELM_NO_TUNE") != nullptr;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  const int r0 = min_rounds<T>(bpmax), nmt = bpmax / 16;
  if (tv.rg == 0 && !no_tune && may_tune && cap == hipStreamCaptureStatusNone) {
    // time every admissible (group, rounds) pair twice on this very input (the
    // sweep is idempotent: z and the scratch planes are overwritten) and keep
    // the fastest
    hipEvent_t e0, e1;
    (void)locked_event_create(&e0);
    (void)locked_event_create(&e1);
    float best = 1e30f;
    static const bool verbose = std::getenv("HELM_TUNE_VERBOSE") != nullptr;
    for (int cand = 8; cand <= rgmax; cand *= 2) {
      int last_waves = 0;
      // rounds 0 = the pipelined persistent sweep, then the one-item sweep with
      // r0, r0 + 1, r0 + 2 tile rounds per wave (and, where it exists, its
      // two-workgroups-per-CU build at r0)
      for (int rounds = 0; rounds <= r0 + 2; rounds = rounds == 0 ? r0 : rounds + 1) {
        if (rounds == 0 && (!allow_pipe || !pipe_fits<T>(cand, bpmax))) continue;
        if (rounds != 0 && !allow_item) continue;
        const int waves = rounds == 0 ? -1 : (nmt + rounds - 1) / rounds;
        if (waves == last_waves) continue;
        last_waves = waves;
        for (int lr = 0; lr < 3; ++lr) {
          // lr 1: the 16-wave pipelined build, or the FP64 32-group build for two workgroups per CU;
          // lr 2: the one-group sweep with its plane solutions in LDS
          if (lr == 1 && !(rounds == 0 || (rounds == r0 && lowreg_fits<T>(cand, bpmax)))) continue;
          if (lr == 2 && !(rounds != 0 && (policy == 0 || policy == 6) && item_ylds_fits<T>(cand, bpmax))) continue;
          float tot = 0.f;
          for (int rep = 0; rep < 2; ++rep) {
            (void)hipEventRecord(e0, s);
            launch_rg<T>(cand, rounds, lr == 1, lr == 2 ? 2 : 0, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny,
                         yloc, tbuf, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) tot += ms;
          }
          if (verbose)
            std::fprintf(stderr, "helm:   candidate group %d %s %d waves%s: %.3f ms\n", cand,
                         rounds == 0 ? "pipelined," : "", rounds == 0 ? (lr ? 16 : 12) : waves,
                         lr == 1 && rounds != 0 ? " (two per CU)" : (lr == 2 ? " (solutions in LDS)" : ""), tot);
          if (tot < best) {
            best = tot;
            tv = {cand, rounds, lr == 1, lr == 2 ? 2 : 0};
          }
        }
      }
      // the paired sweep: two groups of a box per workgroup
      for (int pm = 1; pm <= 2; ++pm) {
        if (!(policy == 0 || policy == 5 || policy == 6) || !pair_fits<T>(cand, bpmax, nrhs)) break;
        if (pm == 2 && !pair_ylds_fits<T>(cand, bpmax, nrhs)) break;
        const int pr0 = pair_min_rounds<T>(bpmax);
        int last = 0;
        for (int rounds = pr0; rounds <= pr0 + 2; ++rounds) {
          const int waves = (nmt + rounds - 1) / rounds;
          if (waves == last) continue;
          last = waves;
          float tot = 0.f;
          for (int rep = 0; rep < 2; ++rep) {
            (void)hipEventRecord(e0, s);
            launch_rg<T>(cand, rounds, false, pm == 2 ? 3 : 1, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny,
                         yloc, tbuf, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) tot += ms;
          }
          if (verbose)
            std::fprintf(stderr, "helm:   candidate group %d paired%s, 2 x %d waves: %.3f ms\n", cand,
                         pm == 2 ? " (solutions in LDS)" : "", waves, tot);
          if (tot < best) {
            best = tot;
            tv = {cand, rounds, false, pm == 2 ? 3 : 1};
          }
        }
      }
    }
    locked_event_destroy(e0);
    locked_event_destroy(e1);
    if (verbose)
      std::fprintf(stderr, "helm: sweep tuned (fp%d, bp %d, %d boxes, %d rhs): group %d, %s %d waves%s, %.3f ms\n",
                   (int)sizeof(T) * 8, bpmax, nsub, nrhs, tv.rg,
                   tv.rounds == 0 ? "pipelined,"
                                  : (tv.pair == 3 ? "paired (LDS solutions), 2 x"
                                                  : (tv.pair == 1 ? "paired, 2 x" : (tv.pair == 2 ? "LDS solutions," : ""))),
                   tv.rounds == 0 ? (tv.lowreg ? 16 : 12) : (nmt + tv.rounds - 1) / tv.rounds,
                   tv.lowreg && tv.rounds != 0 ? " (two per CU)" : "", best);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    store_tune_locked(key, tv);
  }
  if (tv.rg == 0) {  // untuned (tuning off, or inside a capture): the widest group
    tv = {rgmax, r0, false, 0};
    if (!allow_item) {
      for (int cand = rgmax; cand >= 16; cand /= 2)
        if (pipe_fits<T>(cand, bpmax)) {
          tv = {cand, 0, false, 0};
          break;
        }
    }
  }
  launch_rg<T>(tv.rg, tv.rounds, tv.lowreg, tv.pair, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc, tbuf, s);
  return true;
}

template bool oras_fused<float>(const Sub*, int, int, const c32*, const c32*, int, const z64*, z64*, const z64*, int,
                                int, c32*, c32*, hipStream_t, bool);
template bool oras_fused<double>(const Sub*, int, int, const z64*, const z64*, int, const z64*, z64*, const z64*, int,
                                 int, z64*, z64*, hipStream_t, bool);
template int fused_group<float>(int, int);
template int fused_group<double>(int, int);

// ---- approximate local solves: launch and tuning ------------------------------

namespace {
template <int RG, bool YLDS = false>
void launch_half_t(const Sub* subs, int nsub, int ngroups, int nrhs, int bpmax, int rounds, const c32* cpl,
                   const uint4* sinv16, const int* sexp, int maxez, const z64* u, z64* z, const z64* add, int gnx,
                   int gny, c32* yloc, hipStream_t s) {
  constexpr int PF = 4;
  const int ys_off = bpmax * lds_width<float>(RG);
  const size_t lds = ((size_t)ys_off + (YLDS ? (size_t)bpmax * RG : 0)) * sizeof(c32);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_oras_half<RG, PF, YLDS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024 - 2 * RG * (int)sizeof(unsigned));
    attr = true;
  }
  const int nmt = bpmax / 16;
  rounds = std::max(rounds, (nmt + 15) / 16);  // at most 16 waves
  const int nwaves = (nmt + rounds - 1) / rounds;
  hipLaunchKernelGGL((k_oras_half<RG, PF, YLDS>), dim3(nsub * ngroups), dim3(64 * nwaves), lds, s, subs, ngroups, nrhs,
                     cpl, sinv16, sexp, maxez, u, z, add, gnx, gny, yloc, ys_off);
}

// The FP16 sweep with its plane solutions in LDS (groups of 16): operand, solutions and column maxima in one CU's LDS.
bool half_ylds_fits(int rg, int bpmax) {
  return rg == 16 && (size_t)bpmax * (lds_width<float>(rg) + rg) * sizeof(c32) <= 160 * 1024 - 2 * rg * sizeof(unsigned);
}

void launch_half_rg(int rg, int rounds, bool ylds, const Sub* subs, int nsub, int nrhs, int bpmax, const c32* cpl,
                    const uint4* sinv16, const int* sexp, int maxez, const z64* u, z64* z, const z64* add, int gnx,
                    int gny, c32* yloc, hipStream_t s) {
  const int ngroups = (nrhs + rg - 1) / rg;
  if (rg == 16 && ylds)
    launch_half_t<16, true>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv16, sexp, maxez, u, z, add, gnx, gny,
                            yloc, s);
  else if (rg == 16)
    launch_half_t<16>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv16, sexp, maxez, u, z, add, gnx, gny, yloc, s);
  else
    launch_half_t<32>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv16, sexp, maxez, u, z, add, gnx, gny, yloc, s);
}
}  // namespace

int half_group(int bpmax, int nrhs) {
  int rg = nrhs <= 16 ? 16 : 32;
  while (rg >= 16 && !lds_fits<float>(rg, bpmax)) rg /= 2;
  return rg >= 16 ? rg : 0;
}

bool oras_half(const Sub* subs, int nsub, int bpmax, const c32* cpl, const uint4* sinv16, const int* sexp, int maxez,
               int nrhs, const z64* u, z64* z, const z64* add, int gnx, int gny, c32* yloc, hipStream_t s,
               bool may_tune) {
  const int rgmax = half_group(bpmax, nrhs);
  if (rgmax == 0) return false;
  const TuneKey key{2, bpmax, nsub, nrhs, gnx, gny, g_sweep_policy.load()};
  TuneVal tv{0, 0, false, 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) tv = it->second;
  }
  const int nmt = bpmax / 16, r0 = (nmt + 15) / 16;
  if (tv.rg != 0 && ((tv.rg != 16 && tv.rg != 32) || tv.rg > rgmax || tv.rounds < r0 || tv.lowreg ||
                     (tv.pair != 0 && !(tv.pair == 2 && half_ylds_fits(tv.rg, bpmax)))))
    tv = TuneVal{0, 0, false, 0};  // a stale or foreign entry
  const int policy = g_sweep_policy.load();
  if (policy == 6 && rgmax >= 16 && half_ylds_fits(16, bpmax)) {  // forced: plane solutions in LDS
    launch_half_rg(16, r0, true, subs, nsub, nrhs, bpmax, cpl, sinv16, sexp, maxez, u, z, add, gnx, gny, yloc, s);
    return true;
  }
  static const bool no_tune = std::getenv("HELM_NO_TUNE") != nullptr;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  if (tv.rg == 0 && !no_tune && may_tune && cap == hipStreamCaptureStatusNone) {
    hipEvent_t e0, e1;
    (void)locked_event_create(&e0);
    (void)locked_event_create(&e1);
    float best = 1e30f;
    static const bool verbose = std::getenv("HELM_TUNE_VERBOSE") != nullptr;
    for (int cand = 16; cand <= rgmax; cand *= 2) {
      int last_waves = 0;
      for (int rounds = r0; rounds <= r0 + 2; ++rounds) {
        const int waves = (nmt + rounds - 1) / rounds;
        if (waves == last_waves) continue;
        last_waves = waves;
        for (int yl = 0; yl < 2; ++yl) {  // yl 1: the plane solutions in LDS
          if (yl && !((policy == 0 || policy == 6) && half_ylds_fits(cand, bpmax))) continue;
          float tot = 0.f;
          for (int rep = 0; rep < 2; ++rep) {
            (void)hipEventRecord(e0, s);
            launch_half_rg(cand, rounds, yl != 0, subs, nsub, nrhs, bpmax, cpl, sinv16, sexp, maxez, u, z, add, gnx, gny,
                           yloc, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) tot += ms;
          }
          if (verbose)
            std::fprintf(stderr, "helm:   fp16 candidate group %d, %d waves%s: %.3f ms\n", cand, waves,
                         yl ? " (solutions in LDS)" : "", tot);
          if (tot < best) {
            best = tot;
            tv = {cand, rounds, false, yl ? 2 : 0};
          }
        }
      }
    }
    locked_event_destroy(e0);
    locked_event_destroy(e1);
    if (verbose)
      std::fprintf(stderr, "helm: fp16 sweep tuned (bp %d, %d boxes, %d rhs): group %d, %d waves%s, %.3f ms\n", bpmax,
                   nsub, nrhs, tv.rg, (nmt + tv.rounds - 1) / tv.rounds, tv.pair == 2 ? " (solutions in LDS)" : "",
                   best);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    store_tune_locked(key, tv);
  }
  if (tv.rg == 0) tv = {rgmax, r0, false, 0};
  launch_half_rg(tv.rg, tv.rounds, tv.pair == 2, subs, nsub, nrhs, bpmax, cpl, sinv16, sexp, maxez, u, z, add, gnx, gny,
                 yloc, s);
  return true;
}

void launch_to_half(const Sub* subs, int nsub, int maxez, const c32* sinv, uint4* sinv16, int* sexp, hipStream_t s) {
  hipLaunchKernelGGL(k_to_half, dim3(maxez, nsub), dim3(256), 0, s, subs, maxez, sinv, sinv16, sexp);
}
