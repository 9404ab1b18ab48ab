// Batched Krylov kernels: one Krylov space per right-hand side, all spaces
// advanced by the same launches (GMRES of the domain-decomposition section,
// taken as right-preconditioned flexible GMRES).  Orthogonalisation is
// classical Gram-Schmidt applied twice (CGS2) with the coefficient sets
// accumulated; rotations are complex Givens rotations
//   G = [[c, s], [-conj(s), c]],  c = |a|/rho,  s = (a/|a|) conj(b)/rho,
// with c = 0, s = 1 when a = 0.
#include "kernels.h"

namespace {

constexpr int NVMAX = 16;  // basis vectors handled by one dot-product / update launch

__global__ void k_fill(z64* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = mk(0.0, 0.0);
}
__global__ void k_copy(const z64* a, z64* b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}
__global__ void k_sub(z64* a, const z64* b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a[i] = a[i] - b[i];
}
__global__ void k_add2(z64* a, const z64* b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a[i] = a[i] + b[i];
}

// [nrhs][len] -> [len][nrhs] through a 32x32 LDS tile
__global__ void k_to_node_major(const z64* __restrict__ in, z64* __restrict__ out, long long len, int nrhs) {
  __shared__ z64 tile[32][33];
  const long long n0 = blockIdx.x * 32LL;
  const int r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k;
    const long long nd = n0 + tx;
    if (r < nrhs && nd < len) tile[k][tx] = in[(long long)r * len + nd];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const long long nd = n0 + k;
    const int r = r0 + tx;
    if (r < nrhs && nd < len) out[nd * nrhs + r] = tile[tx][k];
  }
}
__global__ void k_to_field_major(const z64* __restrict__ in, z64* __restrict__ out, long long len, int nrhs) {
  __shared__ z64 tile[32][33];
  const long long n0 = blockIdx.x * 32LL;
  const int r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const long long nd = n0 + k;
    const int r = r0 + tx;
    if (r < nrhs && nd < len) tile[k][tx] = in[nd * nrhs + r];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k;
    const long long nd = n0 + tx;
    if (r < nrhs && nd < len) out[(long long)r * len + nd] = tile[tx][k];
  }
}

struct Span {
  long long lo, hi;
};
__device__ __forceinline__ Span block_span(long long len) {
  const long long per = (len + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  return {lo, lo + per < len ? lo + per : len};
}

// Block partial sums are stored output-major, partial[(v * nrhs + r) * nblk + blk],
// so that the final reductions read each output's partials contiguously.

// partial[v][r][blk] = sum over the block's nodes of conj(V_v) w; with npart,
// also npart[r][blk] = sum |w|^2 (the norm read along with the projections)
__global__ void __launch_bounds__(256) k_dots(const z64* __restrict__ V, long long vstride, int nv,
                                              const z64* __restrict__ w, long long len, int nrhs,
                                              z64* __restrict__ partial, double* __restrict__ npart) {
  __shared__ z64 red[256];
  __shared__ double nred[256];
  const int tid = threadIdx.x;
  const int nl = 256 / nrhs;
  const int r = tid % nrhs, lane = tid / nrhs;
  const Span sp = block_span(len);
  z64 acc[NVMAX];
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) acc[v] = mk(0.0, 0.0);
  double nacc = 0.0;
  if (lane < nl) {
    for (long long nd = sp.lo + lane; nd < sp.hi; nd += nl) {
      const long long e = nd * nrhs + r;
      const z64 wv = w[e];
      nacc += abs2(wv);
#pragma unroll
      for (int v = 0; v < NVMAX; ++v)
        if (v < nv) cdot_acc(acc[v], V[(long long)v * vstride + e], wv);
    }
  }
  if (npart) {  // uniform over the block
    nred[tid] = (lane < nl) ? nacc : 0.0;
    __syncthreads();
    if (lane == 0) {
      double t = nred[r];
      for (int l = 1; l < nl; ++l) t += nred[l * nrhs + r];
      npart[(long long)r * gridDim.x + blockIdx.x] = t;
    }
  }
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) {
    if (v < nv) {  // uniform over the block
      red[tid] = (lane < nl) ? acc[v] : mk(0.0, 0.0);
      __syncthreads();
      if (lane == 0) {
        z64 s = red[r];
        for (int l = 1; l < nl; ++l) s += red[l * nrhs + r];
        partial[((long long)v * nrhs + r) * gridDim.x + blockIdx.x] = s;
      }
      __syncthreads();
    }
  }
}

// Fixed-order sum over the 64 lanes of a wave (the same tree on every call).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
__device__ __forceinline__ z64 wave_sum(z64 v) { return mk(wave_sum(v.re), wave_sum(v.im)); }

// out[t] = sum_b partial[t][b] for t < nout: one wave per output, lanes over
// the blocks (coalesced), four independent accumulators, fixed order.
__global__ void __launch_bounds__(256) k_dots_final(const z64* __restrict__ partial, int nblk, int nv, int nrhs,
                                                    z64* __restrict__ h) {
  const int nout = nv * nrhs;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= nout) return;
  const z64* p = partial + (long long)t * nblk;
  z64 s[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  int b = lane;
  for (; b + 192 < nblk; b += 256) {
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] += p[b + 64 * i];
  }
  if (b < nblk) s[0] += p[b];
  if (b + 64 < nblk) s[1] += p[b + 64];
  if (b + 128 < nblk) s[2] += p[b + 128];
  const z64 tot = wave_sum((s[0] + s[1]) + (s[2] + s[3]));
  if (lane == 0) h[t] = tot;
}

// w -= sum_v h[v][r] V_v; partial[r][blk] = sum |w|^2 over the block's nodes (if partial)
__global__ void __launch_bounds__(256) k_axpy_multi(const z64* __restrict__ V, long long vstride, int nv,
                                                    const z64* __restrict__ h, z64* __restrict__ w, long long len,
                                                    int nrhs, double* __restrict__ partial,
                                                    const int* __restrict__ skip) {
  if (skip && *skip) return;  // uniform: one flag for the whole launch
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int nl = 256 / nrhs;
  const int r = tid % nrhs, lane = tid / nrhs;
  const Span sp = block_span(len);
  z64 hv[NVMAX];
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) hv[v] = (v < nv) ? h[v * nrhs + r] : mk(0.0, 0.0);
  double acc = 0.0;
  if (lane < nl) {
    for (long long nd = sp.lo + lane; nd < sp.hi; nd += nl) {
      const long long e = nd * nrhs + r;
      z64 x = w[e];
#pragma unroll
      for (int v = 0; v < NVMAX; ++v)
        if (v < nv) cfms(x, hv[v], V[(long long)v * vstride + e]);
      w[e] = x;
      acc += abs2(x);
    }
  }
  if (partial) {
    red[tid] = (lane < nl) ? acc : 0.0;
    __syncthreads();
    if (lane == 0) {
      double s = red[r];
      for (int l = 1; l < nl; ++l) s += red[l * nrhs + r];
      partial[(long long)r * gridDim.x + blockIdx.x] = s;
    }
  }
}

// Fused CGS pass: w -= sum_v h[v][r] V_v, then partial[v][r][blk] = sum conj(V_v) w
// over the block's nodes -- the update of the first Gram-Schmidt pass and the
// projections of the second in one read of the basis.
// nv vectors update w; the first ndot <= NVMAX of them also take the projections
// (the rest, if any, by a separate dot-product launch on the updated w).
__global__ void __launch_bounds__(256) k_axpy_dots(const z64* __restrict__ V, long long vstride, int nv, int ndot,
                                                   const z64* __restrict__ h, z64* __restrict__ w, long long len,
                                                   int nrhs, z64* __restrict__ partial, double* __restrict__ npart) {
  extern __shared__ z64 hs[];  // [nv][nrhs]
  __shared__ z64 red[256];
  const int tid = threadIdx.x;
  for (int t = tid; t < nv * nrhs; t += 256) hs[t] = h[t];
  __syncthreads();
  const int nl = 256 / nrhs;
  const int r = tid % nrhs, lane = tid / nrhs;
  const Span sp = block_span(len);
  z64 acc[NVMAX];
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) acc[v] = mk(0.0, 0.0);
  double accn = 0.0;
  if (lane < nl) {
    for (long long nd = sp.lo + lane; nd < sp.hi; nd += nl) {
      const long long e = nd * nrhs + r;
      z64 x = w[e];
      z64 vv[NVMAX];
#pragma unroll
      for (int v = 0; v < NVMAX; ++v)
        if (v < ndot) {
          vv[v] = V[(long long)v * vstride + e];
          cfms(x, hs[v * nrhs + r], vv[v]);
        }
      for (int v = ndot; v < nv; ++v) cfms(x, hs[v * nrhs + r], V[(long long)v * vstride + e]);
      w[e] = x;
      accn += abs2(x);
#pragma unroll
      for (int v = 0; v < NVMAX; ++v)
        if (v < ndot) cdot_acc(acc[v], vv[v], x);
    }
  }
  if (npart) {  // ||w'||^2 partial, [r][blk] as k_norm2 (red reused as doubles after a barrier)
    double* rd = reinterpret_cast<double*>(red);
    rd[tid] = (lane < nl) ? accn : 0.0;
    __syncthreads();
    if (lane == 0) {
      double sn = rd[r];
      for (int l = 1; l < nl; ++l) sn += rd[l * nrhs + r];
      npart[(long long)r * gridDim.x + blockIdx.x] = sn;
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) {
    if (v < ndot) {  // uniform over the block
      red[tid] = (lane < nl) ? acc[v] : mk(0.0, 0.0);
      __syncthreads();
      if (lane == 0) {
        z64 sacc = red[r];
        for (int l = 1; l < nl; ++l) sacc += red[l * nrhs + r];
        partial[((long long)v * nrhs + r) * gridDim.x + blockIdx.x] = sacc;
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(256) k_norm2(const z64* __restrict__ w, long long len, int nrhs,
                                               double* __restrict__ partial) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int nl = 256 / nrhs;
  const int r = tid % nrhs, lane = tid / nrhs;
  const Span sp = block_span(len);
  double acc = 0.0;
  if (lane < nl)
#pragma unroll 4
    for (long long nd = sp.lo + lane; nd < sp.hi; nd += nl) acc += abs2(w[nd * nrhs + r]);
  red[tid] = (lane < nl) ? acc : 0.0;
  __syncthreads();
  if (lane == 0) {
    double s = red[r];
    for (int l = 1; l < nl; ++l) s += red[l * nrhs + r];
    partial[(long long)r * gridDim.x + blockIdx.x] = s;
  }
}

// out[r] = sum_b partial[r][b]: one wave per output, as k_dots_final.
__global__ void __launch_bounds__(256) k_sum_final(const double* __restrict__ partial, int nblk, int nrhs,
                                                   double* __restrict__ out, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= nrhs) return;
  const double* p = partial + (long long)r * nblk;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int b = lane;
  for (; b + 192 < nblk; b += 256) {
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] += p[b + 64 * i];
  }
  if (b < nblk) s[0] += p[b];
  if (b + 64 < nblk) s[1] += p[b + 64];
  if (b + 128 < nblk) s[2] += p[b + 128];
  const double tot = wave_sum((s[0] + s[1]) + (s[2] + s[3]));
  if (lane == 0) out[r] = tot;
}

__global__ void k_scale(const z64* __restrict__ w, const double* __restrict__ fac, z64* __restrict__ out,
                        long long len, int nrhs) {
  const long long n = len * nrhs;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = fac[e % nrhs] * w[e];
}

__global__ void k_update(const z64* __restrict__ Z, long long zstride, int nv, const z64* __restrict__ y,
                         z64* __restrict__ x, long long len, int nrhs) {
  const long long n = len * nrhs;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % nrhs);
    z64 acc = x[e];
    for (int v = 0; v < nv; ++v) cfma(acc, y[v * nrhs + r], Z[(long long)v * zstride + e]);
    x[e] = acc;
  }
}

__global__ void k_krylov_init(KrylovState st, const double* __restrict__ bn2) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= st.nrhs) return;
  st.bnorm[r] = sqrt(bn2[r]);
  st.it[r] = 0;
  st.kc[r] = 0;
  st.active[r] = 0;
  st.done[r] = 0;
  st.conv[r] = 0;
  st.est[r] = 1.0;
}

// Outer cycle start from the current residual norm^2 (beta2): done when
// ||r|| <= tol ||b|| (converged) or it >= maxit; else v_0 = r/||r||.
__global__ void k_cycle_start(KrylovState st, const double* __restrict__ beta2, double tol, int maxit, int first) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= st.nrhs) return;
  st.kc[r] = 0;
  if (st.done[r]) {
    st.active[r] = 0;
    st.fac[r] = 0.0;
    return;
  }
  const double beta = sqrt(beta2[r]);
  const double bn = st.bnorm[r];
  st.beta[r] = beta;
  if (first) st.est[r] = bn > 0.0 ? beta / bn : 0.0;
  if (bn == 0.0 || beta <= tol * bn || st.it[r] >= maxit) {
    st.done[r] = 1;
    st.conv[r] = (bn == 0.0 || beta <= tol * bn) ? 1 : 0;
    st.active[r] = 0;
    st.fac[r] = 0.0;
    return;
  }
  st.g[r] = mk(beta, 0.0);
  st.fac[r] = 1.0 / beta;
  st.active[r] = 1;
  atomicAdd(st.counter, 1);
}

// Fixed-length (coarse) GMRES from x0 = 0: v_0 = c/||c||, nothing to do when c = 0.
__global__ void k_cycle_start_fixed(KrylovState st, const double* __restrict__ beta2) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= st.nrhs) return;
  st.kc[r] = 0;
  const double beta = sqrt(beta2[r]);
  if (beta == 0.0) {
    st.active[r] = 0;
    st.fac[r] = 0.0;
    return;
  }
  st.g[r] = mk(beta, 0.0);
  st.fac[r] = 1.0 / beta;
  st.active[r] = 1;
}

__global__ void k_givens(KrylovState st, int j, double tol, int maxit, int fixed) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= st.nrhs) return;
  const int nr = st.nrhs;
  if (!st.active[r]) {
    st.fac[r] = 0.0;
    return;
  }
  const double hnext = sqrt(st.nrm2[r]);
  // rotate the new column h[0..j], hnext by the previous rotations
  // coefficients of the two Gram-Schmidt passes, accumulated
  z64 a = st.h[r] + st.h2[r];
  for (int i = 0; i < j; ++i) {
    const z64 b = st.h[(i + 1) * nr + r] + st.h2[(i + 1) * nr + r];
    const double c = st.cs[i * nr + r];
    const z64 s = st.sn[i * nr + r];
    const z64 top = c * a + s * b;
    const z64 bot = c * b - conj(s) * a;
    st.Rm[((long long)i * st.m + j) * nr + r] = top;
    a = bot;
  }
  // new rotation on (a, hnext)
  const z64 bb = mk(hnext, 0.0);
  double c;
  z64 s, rho;
  const double aa = sqrt(abs2(a));
  if (aa == 0.0) {
    c = 0.0;
    s = mk(1.0, 0.0);
    rho = bb;
  } else {
    const double nrm = sqrt(aa * aa + hnext * hnext);
    const z64 ph = (1.0 / aa) * a;
    c = aa / nrm;
    s = (1.0 / nrm) * (ph * conj(bb));
    rho = nrm * ph;
  }
  st.cs[j * nr + r] = c;
  st.sn[j * nr + r] = s;
  st.Rm[((long long)j * st.m + j) * nr + r] = rho;
  const z64 gj = st.g[j * nr + r];
  st.g[(j + 1) * nr + r] = -(conj(s) * gj);
  st.g[j * nr + r] = c * gj;
  st.kc[r] = j + 1;
  bool stop = hnext <= 1e-14 * sqrt(st.w0[r]) || j + 1 >= st.m;
  if (!fixed) {
    const double est = sqrt(abs2(st.g[(j + 1) * nr + r])) / st.bnorm[r];
    st.it[r] += 1;
    st.est[r] = est;
    stop = stop || est <= tol || st.it[r] >= maxit;
  }
  if (stop) {
    st.active[r] = 0;
    st.fac[r] = 0.0;
  } else {
    st.fac[r] = 1.0 / hnext;
    atomicAdd(st.counter, 1);
  }
}

// y = R^{-1} g over the kc steps of the current cycle (zero beyond)
__global__ void k_backsolve(KrylovState st) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= st.nrhs) return;
  const int nr = st.nrhs;
  const int k = st.kc[r];
  for (int i = st.m - 1; i >= 0; --i) {
    if (i >= k) {
      st.y[i * nr + r] = mk(0.0, 0.0);
      continue;
    }
    z64 acc = st.g[i * nr + r];
    for (int l = i + 1; l < k; ++l) cfms(acc, st.Rm[((long long)i * st.m + l) * nr + r], st.y[l * nr + r]);
    st.y[i * nr + r] = cdiv(acc, st.Rm[((long long)i * st.m + i) * nr + r]);
  }
}

int red_blocks(long long len) {
  long long b = ceil_div(len, 256);
  if (b < 1) b = 1;
  if (b > RED_BLOCKS) b = RED_BLOCKS;
  return (int)b;
}

}  // namespace

void launch_fill(z64* p, long long n, hipStream_t s) {
  account(16.0 * n, 0);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<long long>(ceil_div(n, 256), 8192)), dim3(256), 0, s, p, n);
}
void launch_copy(const z64* a, z64* b, long long n, hipStream_t s) {
  account(32.0 * n, 0);
  hipLaunchKernelGGL(k_copy, dim3((unsigned)std::min<long long>(ceil_div(n, 256), 8192)), dim3(256), 0, s, a, b, n);
}
void launch_sub(z64* a, const z64* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3((unsigned)std::min<long long>(ceil_div(n, 256), 8192)), dim3(256), 0, s, a, b, n);
}
void launch_add2(z64* a, const z64* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_add2, dim3((unsigned)std::min<long long>(ceil_div(n, 256), 8192)), dim3(256), 0, s, a, b, n);
}
void launch_to_node_major(const z64* in, z64* out, long long len, int nrhs, hipStream_t s) {
  account(32.0 * len * nrhs, 0);
  hipLaunchKernelGGL(k_to_node_major, dim3((unsigned)ceil_div(len, 32), (unsigned)ceil_div(nrhs, 32)), dim3(256), 0, s,
                     in, out, len, nrhs);
}
// out[i][c] = in[i][cols[c]]: selected columns of a node-major block ([len][nin] -> [len][nout])
__global__ void k_gather_cols(const z64* __restrict__ in, int nin, const int* __restrict__ cols, int nout,
                              long long len, z64* __restrict__ out) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= len * nout) return;
  const long long i = e / nout;
  const int c = (int)(e - i * nout);
  out[e] = in[i * nin + cols[c]];
}
void launch_gather_cols(const z64* in, int nin, const int* cols, int nout, long long len, z64* out, hipStream_t s) {
  account(32.0 * len * nout, 0);
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)ceil_div(len * nout, 256)), dim3(256), 0, s, in, nin, cols, nout,
                     len, out);
}

void launch_to_field_major(const z64* in, z64* out, long long len, int nrhs, hipStream_t s) {
  account(32.0 * len * nrhs, 0);
  hipLaunchKernelGGL(k_to_field_major, dim3((unsigned)ceil_div(len, 32), (unsigned)ceil_div(nrhs, 32)), dim3(256), 0,
                     s, in, out, len, nrhs);
}

void launch_dots(const z64* V, long long vstride, int nv, const z64* w, long long len, int nrhs, z64* partial,
                 z64* h, hipStream_t s, double* npart, double* nrm2) {
  account(16.0 * (nv + 1) * len * nrhs, 8.0 * nv * len * nrhs);
  const int nblk = red_blocks(len);
  for (int v0 = 0; v0 < nv; v0 += NVMAX) {
    const int nvb = std::min(NVMAX, nv - v0);
    double* np = (v0 == 0 && nrm2) ? npart : nullptr;
    hipLaunchKernelGGL(k_dots, dim3(nblk), dim3(256), 0, s, V + v0 * vstride, vstride, nvb, w, len, nrhs, partial,
                       np);
    if (np)
      hipLaunchKernelGGL(k_sum_final, dim3((unsigned)ceil_div(nrhs, 4)), dim3(256), 0, s, np, nblk, nrhs, nrm2,
                         (const int*)nullptr);
    hipLaunchKernelGGL(k_dots_final, dim3((unsigned)ceil_div(nvb * nrhs, 4)), dim3(256), 0, s, partial, nblk, nvb,
                       nrhs, h + (long long)v0 * nrhs);
  }
}

void launch_axpy_multi(const z64* V, long long vstride, int nv, const z64* h, z64* w, long long len, int nrhs,
                       double* partial, double* nrm2, hipStream_t s, const int* skip) {
  // a conditional update is accounted on the device, when it runs (launch_reorth_check)
  if (!skip) account(16.0 * (nv + 2) * len * nrhs, 8.0 * nv * len * nrhs);
  const int nblk = red_blocks(len);
  for (int v0 = 0; v0 < nv; v0 += NVMAX) {
    const int nvb = std::min(NVMAX, nv - v0);
    const bool last = v0 + nvb >= nv;
    hipLaunchKernelGGL(k_axpy_multi, dim3(nblk), dim3(256), 0, s, V + v0 * vstride, vstride, nvb,
                       h + (long long)v0 * nrhs, w, len, nrhs, (last && nrm2) ? partial : nullptr, skip);
  }
  if (nrm2)
    hipLaunchKernelGGL(k_sum_final, dim3((unsigned)ceil_div(nrhs, 4)), dim3(256), 0, s, partial, nblk, nrhs, nrm2,
                       skip);
}

// One workgroup; each thread owns right-hand sides r = tid, tid + 256, ...
__global__ void __launch_bounds__(256) k_reorth_check(KrylovState st, int nv, double tau2, double vec_bytes) {
  const int nr = st.nrhs;
  int need = 0;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    if (!st.active[r]) continue;
    double s2 = 0.0;
    for (int v = 0; v < nv; ++v) s2 += abs2(st.h2[v * nr + r]);
    if (s2 > tau2 * st.w1[r]) need = 1;
  }
  const int any = __syncthreads_or(need);
  if (!any) {
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
      for (int v = 0; v < nv; ++v) st.h2[v * nr + r] = mk(0.0, 0.0);
      st.nrm2[r] = st.w1[r];
    }
  } else if (threadIdx.x == 0) {
    atomicAdd(st.extra, vec_bytes * (nv + 2));
  }
  if (threadIdx.x == 0) *st.skip = any ? 0 : 1;
}
void launch_reorth_check(KrylovState st, int nv, double tau2, double vec_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_reorth_check, dim3(1), dim3(256), 0, s, st, nv, tau2, vec_bytes);
}

bool launch_axpy_dots(const z64* V, long long vstride, int nv, const z64* h, z64* w, long long len, int nrhs,
                      z64* partial, z64* h2, hipStream_t s, double* npart, double* nrm2) {
  if ((size_t)nv * nrhs * sizeof(z64) > 64 * 1024) return false;
  // the update and the first NVMAX projections in one pass; projections on
  // further vectors (restart lengths above NVMAX) read the updated w once more
  const int nd = std::min(nv, NVMAX);
  account(16.0 * (nv + 2) * len * nrhs, 8.0 * (nv + nd) * len * nrhs);  // launch_dots accounts its own pass
  const int nblk = red_blocks(len);
  hipLaunchKernelGGL(k_axpy_dots, dim3(nblk), dim3(256), (size_t)nv * nrhs * sizeof(z64), s, V, vstride, nv, nd, h, w,
                     len, nrhs, partial, nrm2 ? npart : nullptr);
  if (nrm2)
    hipLaunchKernelGGL(k_sum_final, dim3((unsigned)ceil_div(nrhs, 4)), dim3(256), 0, s, npart, nblk, nrhs, nrm2,
                       (const int*)nullptr);
  hipLaunchKernelGGL(k_dots_final, dim3((unsigned)ceil_div(nd * nrhs, 4)), dim3(256), 0, s, partial, nblk, nd, nrhs,
                     h2);
  if (nv > nd) launch_dots(V + (long long)nd * vstride, vstride, nv - nd, w, len, nrhs, partial, h2 + (long long)nd * nrhs, s);
  return true;
}

void launch_norm2(const z64* w, long long len, int nrhs, double* partial, double* nrm2, hipStream_t s) {
  account(16.0 * len * nrhs, 4.0 * len * nrhs);
  const int nblk = red_blocks(len);
  hipLaunchKernelGGL(k_norm2, dim3(nblk), dim3(256), 0, s, w, len, nrhs, partial);
  hipLaunchKernelGGL(k_sum_final, dim3((unsigned)ceil_div(nrhs, 4)), dim3(256), 0, s, partial, nblk, nrhs, nrm2,
                     (const int*)nullptr);
}

void launch_scale(const z64* w, const double* fac, z64* out, long long len, int nrhs, hipStream_t s) {
  account(32.0 * len * nrhs, 2.0 * len * nrhs);
  hipLaunchKernelGGL(k_scale, dim3((unsigned)std::min<long long>(ceil_div(len * nrhs, 256), 8192)), dim3(256), 0, s,
                     w, fac, out, len, nrhs);
}

void launch_update(const z64* Z, long long zstride, int nv, const z64* y, z64* x, long long len, int nrhs,
                   hipStream_t s) {
  account(16.0 * (nv + 2) * len * nrhs, 8.0 * nv * len * nrhs);
  hipLaunchKernelGGL(k_update, dim3((unsigned)std::min<long long>(ceil_div(len * nrhs, 256), 8192)), dim3(256), 0, s,
                     Z, zstride, nv, y, x, len, nrhs);
}

void launch_krylov_init(KrylovState st, const double* bn2, hipStream_t s) {
  hipLaunchKernelGGL(k_krylov_init, dim3((unsigned)ceil_div(st.nrhs, 64)), dim3(64), 0, s, st, bn2);
}
void launch_cycle_start(KrylovState st, const double* beta2, double tol, int maxit, int first, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_start, dim3((unsigned)ceil_div(st.nrhs, 64)), dim3(64), 0, s, st, beta2, tol, maxit,
                     first);
}
void launch_cycle_start_fixed(KrylovState st, const double* beta2, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_start_fixed, dim3((unsigned)ceil_div(st.nrhs, 64)), dim3(64), 0, s, st, beta2);
}
void launch_givens(KrylovState st, int j, double tol, int maxit, int fixed, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, dim3((unsigned)ceil_div(st.nrhs, 64)), dim3(64), 0, s, st, j, tol, maxit, fixed);
}
void launch_backsolve(KrylovState st, hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve, dim3((unsigned)ceil_div(st.nrhs, 64)), dim3(64), 0, s, st);
}

// ---- block Krylov kernels (block FGMRES) ------------------------------------
//
// Block vectors are batches of s <= 32 right-hand sides, node-major
// (element (node, a) at node * s + a).  Small s x s coefficient blocks are
// stored padded, [block][32][32].

namespace {

constexpr int BK_TILE = 32;  // nodes per LDS tile

// partial[ch][i][a][b] = sum over the nodes of chunk ch of conj(V_i[node][a]) W[node][b].
// 256 threads: four groups of 64, group g takes the tile's nodes g, g + 4, ...;
// lane l of a group owns the 4 x 4 block a = 4 (l / 8) + x, b = 4 (l % 8) + y.
__global__ void __launch_bounds__(256) k_bdot(const z64* __restrict__ V, long long vstride, const z64* __restrict__ W,
                                              long long len, int s, z64* __restrict__ partial) {
  __shared__ z64 sv[BK_TILE][33], sw[BK_TILE][33];
  __shared__ z64 red[32][33];
  const int i = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
  const z64* Vi = V + i * vstride;
  const long long per = ceil_div(len, nch);
  const long long n0 = ch * per, n1 = min(len, n0 + per);
  const int t = threadIdx.x, g = t >> 6, l = t & 63, a0 = 4 * (l >> 3), b0 = 4 * (l & 7);
  z64 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = mk(0.0, 0.0);
  for (long long base = n0; base < n1; base += BK_TILE) {
    const int nt = (int)min((long long)BK_TILE, n1 - base);
    for (int e = t; e < BK_TILE * 32; e += 256) {
      const int q = e >> 5, c = e & 31;
      const bool in = q < nt && c < s;
      sv[q][c] = in ? Vi[(base + q) * s + c] : mk(0.0, 0.0);
      sw[q][c] = in ? W[(base + q) * s + c] : mk(0.0, 0.0);
    }
    __syncthreads();
    for (int q = g; q < BK_TILE; q += 4) {
      z64 va[4], wb[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) va[x] = sv[q][a0 + x];
#pragma unroll
      for (int y = 0; y < 4; ++y) wb[y] = sw[q][b0 + y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) cdot_acc(acc[x][y], va[x], wb[y]);
    }
    __syncthreads();
  }
  // sum the four groups in a fixed order: 0 + 1 + 2 + 3
  for (int gg = 1; gg < 4; ++gg) {
    if (g == gg)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) red[a0 + x][b0 + y] = acc[x][y];
    __syncthreads();
    if (g == 0)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += red[a0 + x][b0 + y];
    __syncthreads();
  }
  if (g == 0) {
    z64* out = partial + ((long long)ch * gridDim.y + i) * 1024;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) out[(a0 + x) * 32 + b0 + y] = acc[x][y];
  }
}

// C[i][a][b] = sum over chunks, in chunk order, of partial[ch][i][a][b].
__global__ void k_bdot_reduce(const z64* __restrict__ partial, int nch, int nv, z64* __restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nv * 1024) return;
  z64 acc = mk(0.0, 0.0);
  for (int ch = 0; ch < nch; ++ch) acc += partial[(long long)ch * nv * 1024 + e];
  C[e] = acc;
}

// out[node][b] = (accumulate ? out[node][b] : 0) + sign sum_{i < nv} sum_{a < s} In_i[node][a] C[i][a][b].
// 256 threads per tile of 32 nodes: thread t owns node t / 8 and the four columns b = 4 (t % 8) + y.
__global__ void __launch_bounds__(256) k_bgemm(const z64* __restrict__ In, long long istride, int nv,
                                               const z64* __restrict__ C, long long len, int s, double sign,
                                               int accumulate, z64* __restrict__ out) {
  __shared__ z64 si[BK_TILE][33], cs[32][33];
  const long long base = (long long)blockIdx.x * BK_TILE;
  const int t = threadIdx.x, nl = t >> 3, b0 = 4 * (t & 7);
  const long long node = base + nl;
  const int nt = (int)min((long long)BK_TILE, len - base);
  z64 acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = mk(0.0, 0.0);
  for (int i = 0; i < nv; ++i) {
    const z64* Ii = In + i * istride;
    for (int e = t; e < BK_TILE * 32; e += 256) {
      const int q = e >> 5, c = e & 31;
      si[q][c] = (q < nt && c < s) ? Ii[(base + q) * s + c] : mk(0.0, 0.0);
      cs[q][c] = C[(long long)i * 1024 + e];
    }
    __syncthreads();
    for (int a = 0; a < s; ++a) {
      const z64 v = si[nl][a];
#pragma unroll
      for (int y = 0; y < 4; ++y) cfma(acc[y], v, cs[a][b0 + y]);
    }
    __syncthreads();
  }
  if (nl < nt) {
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int b = b0 + y;
      if (b >= s) continue;
      z64* o = out + node * s + b;
      const z64 d = mk(sign * acc[y].re, sign * acc[y].im);
      *o = accumulate ? *o + d : d;
    }
  }
}

}  // namespace

int block_chunks(long long len) { return (int)std::min<long long>(std::max<long long>(ceil_div(len, 8192), 1), 240); }

void launch_block_dots(const z64* V, long long vstride, int nv, const z64* W, long long len, int s, z64* partial,
                       z64* C, hipStream_t st) {
  const int nch = block_chunks(len);
  account(16.0 * (nv + 1) * len * s, 8.0 * nv * len * (double)s * s);
  hipLaunchKernelGGL(k_bdot, dim3(nch, nv), dim3(256), 0, st, V, vstride, W, len, s, partial);
  hipLaunchKernelGGL(k_bdot_reduce, dim3((unsigned)ceil_div((long long)nv * 1024, 256)), dim3(256), 0, st, partial, nch,
                     nv, C);
}

void launch_block_gemm(const z64* In, long long istride, int nv, const z64* C, long long len, int s, double sign,
                       bool accumulate, z64* out, hipStream_t st) {
  account(16.0 * (nv + (accumulate ? 2 : 1)) * len * s, 8.0 * nv * len * (double)s * s);
  hipLaunchKernelGGL(k_bgemm, dim3((unsigned)ceil_div(len, BK_TILE)), dim3(256), 0, st, In, istride, nv, C, len, s, sign,
                     accumulate ? 1 : 0, out);
}
