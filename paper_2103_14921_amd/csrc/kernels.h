// Kernel launchers of the HIP library (host-callable).  Vectors are batches
// laid out node-major, right-hand side fastest: element (node, r) at
// node*nrhs + r, complex interleaved.
#pragma once
#include <mutex>

#include "common.h"

// Runtime objects -- streams, events, executable graphs -- are created and
// destroyed under one process-wide lock, which stream capture also holds
// (helm_api.hip): no thread creates or destroys one while another records a
// graph.  Handles take their streams from a pool that never destroys them.
std::recursive_mutex& capture_lock();
hipError_t locked_event_create(hipEvent_t* e);
void locked_event_destroy(hipEvent_t e);

// ---- medium and operator (ops_operator.hip) --------------------------------
struct AxisPml {
  int n, lo, hi;  // nodes, PML thickness at the low / high end
};
// Lower bound of the solve: every launch of the solve phase adds its
// algorithmic bytes and flops and the time they take at the device's peaks
// (HBM 8 TB/s; FP64 78.6, FP32 157.3, dense FP16 matrix 2500 TFLOP/s), into the accumulator the
// calling thread has installed (none outside solves).
struct WorkBound {
  double bytes = 0, flops = 0, seconds = 0;
  void add(const WorkBound& o) {
    bytes += o.bytes;
    flops += o.flops;
    seconds += o.seconds;
  }
};
constexpr double HBM_PEAK = 8.0e12, FP64_PEAK = 78.6e12, FP32_PEAK = 157.3e12, FP16_PEAK = 2.5e15;
extern thread_local WorkBound* g_work;
inline void account(double bytes, double flops, double peak = FP64_PEAK) {
  if (WorkBound* w = g_work) {
    w->bytes += bytes;
    w->flops += flops;
    w->seconds += bytes / HBM_PEAK > flops / peak ? bytes / HBM_PEAK : flops / peak;
  }
}

void launch_vmax(const z64* c, long long n, double* out, hipStream_t s);
void launch_pml_tables(const AxisPml ax[3], double h, double omega, double R, const double* vmax,
                       z64* xi_int, z64* xi_half, z64* i2_int, z64* i2_half, uint8_t* flat,
                       hipStream_t s);
void launch_sigma(const OpDev& op, const z64* c, double omega, hipStream_t s);
// Row diagonals A[i, i] into diag[n] (OpDev::diag), after sigma and the node weights.
void launch_row_diag(const OpDev& op, z64* diag, hipStream_t s);
// Per-node weights of the adaptive coefficients (OpDev::wnode, 8 doubles per
// node) from the weight table tab[ntab][7] at G = g0 + j dg.
void launch_node_weights(const z64* c, long long n, double freq, double h, const double* tab, int ntab, double g0,
                         double dg, double* wnode, hipStream_t s);
// y = A x; y aliases neither x nor b (the first application of a shape outside
// a capture is run several times by the autotuner).
void launch_stencil(const OpDev& op, int nrhs, const z64* x, z64* y, hipStream_t s);
// y = b - A x
void launch_residual(const OpDev& op, int nrhs, const z64* b, const z64* x, z64* y, hipStream_t s);
// True while the row-tiled product for this grid and batch has not been timed
// (an application outside a stream capture times it).
bool stencil_untuned(const OpDev& op, int nrhs);
bool coarse_spmv_untuned(int ncx, int ncy, int ncz, int nrhs);
// Nodes per thread of the row-tiled products: 0 = autotuned, else 2, 4 or 8.
bool set_row_tiling(int nxt);
void launch_build_E(const OpDev& op, int ncx, int ncy, int ncz, z64* E, hipStream_t s);
void launch_coarse_spmv(int ncx, int ncy, int ncz, const z64* E, int nrhs, const z64* x, z64* y,
                        hipStream_t s);
void launch_restrict(int nx, int ny, int nz, int nrhs, const z64* r, z64* c, hipStream_t s);
void launch_prolong(int nx, int ny, int nz, int nrhs, const z64* c, z64* q, hipStream_t s);

// ---- local operators, factorisation and sweeps (ops_local.hip) -------------
// Local operator rows: aloc[(node_off + l)*27 + o], o = (oz+1)*9 + (oy+1)*3 + (ox+1).
void launch_local_fine(const OpDev& op, const Sub* subs, int nsub, long long maxnodes,
                       const z64* c, double omega, double h, int robin, z64* aloc, hipStream_t s);
void launch_local_coarse(int ncx, int ncy, int ncz, const z64* E, const Sub* subs, int nsub,
                         long long maxnodes, const z64* c_fine, int nx, int ny, double omega,
                         double hc, int robin, z64* aloc, hipStream_t s);

// one box: scatter a local field into a zeroed global field / read back the stored plane solutions
void launch_box_scatter(const Sub& sb, int gnx, int gny, int nrhs, const z64* rl, z64* u, hipStream_t s);
template <typename T>
void launch_box_gather(const Sub& sb, int nrhs, const cpx<T>* yloc, z64* xl, hipStream_t s);

// Plane couplings [node][18] (taps to plane k-1, then to plane k+1) in the
// factor precision, extracted from the local operator rows.
template <typename T>
void launch_couplings(long long nodes, const z64* aloc, cpx<T>* cpl, hipStream_t s);

template <typename T>
struct Factor {
  // one plane step of the block-tridiagonal LU: S_k = D_k - L_k Sinv_{k-1} U_{k-1}, Sinv_k = S_k^{-1}
  // Rbuf: [nsub][16][bpmax] panel pivot rows; R64: [nsub][64][bpmax] block pivot rows
  static void plane(const Sub* subs, int nsub, int bpmax, int k, const z64* aloc, cpx<T>* sinv,
                    cpx<T>* W, cpx<T>* S, cpx<T>* Rbuf, cpx<T>* R64, int* piv, int* perm, int* err,
                    hipStream_t s);
  // one application of the batched local solves on all subdomains:
  // z = sum_i R_i^T D_i A_i^{-1} R_i u  (+ add if add != nullptr)
  // may_tune = false: an untuned shape takes the default launch shape instead of
  // timing the candidates (the tuner creates events and synchronises)
  static void sweep(const Sub* subs, int nsub, int bpmax, int maxez, const cpx<T>* cpl,
                    const cpx<T>* sinv, int nrhs, const z64* u, z64* z, const z64* add,
                    int gnx, int gny, cpx<T>* yloc, cpx<T>* tbuf, hipStream_t s, bool may_tune = true);
};

// Panel width (columns) of the blocked Gauss-Jordan plane inversion: 0 =
// autotuned per shape, else 4, 8 or 16 wherever admissible for the plane size.
bool set_lu_panel(int nb);

// Fused single-launch ORAS local solves on matrix cores (ops_sweep.hip).
// Planes whose operand does not fit in LDS keep it in tbuf (at least
// sweep_tbuf_elems elements); returns false for them when tbuf is null.
template <typename T>
bool oras_fused(const Sub* subs, int nsub, int bpmax, const cpx<T>* cpl, const cpx<T>* sinv, int nrhs, const z64* u,
                z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc, cpx<T>* tbuf, hipStream_t s,
                bool may_tune = true);
template <typename T>
int fused_group(int bpmax, int nrhs);
// Elements of the sweeps' operand buffer for nsub boxes of planes up to bpmax
// and nrhs right-hand sides: the per-plane path's [nsub][bpmax][nrhs] and the
// global-operand sweep's [nsub * ceil(nrhs / 8)][bpmax][16].
inline long long sweep_tbuf_elems(int nsub, int bpmax, int nrhs) {
  return (long long)nsub * bpmax * 2 * ((nrhs + 7) / 8 * 8);
}
// Approximate local solves (the FP16 sweep k_oras_half): plane inverses
// converted from complex FP32 by launch_to_half into 16-byte blocks (four real
// parts, four imaginary parts of one row) scaled by 2^-sexp[id * maxez + k]
// (id = the box's Sub::id, so the boxes may be passed in any order).
// oras_half returns false where the complex-FP32 operand of a plane does not
// fit in LDS (half_group 0: planes above 960 nodes).
int half_group(int bpmax, int nrhs);
bool oras_half(const Sub* subs, int nsub, int bpmax, const c32* cpl, const uint4* sinv16, const int* sexp, int maxez,
               int nrhs, const z64* u, z64* z, const z64* add, int gnx, int gny, c32* yloc, hipStream_t s,
               bool may_tune = true);
void launch_to_half(const Sub* subs, int nsub, int maxez, const c32* sinv, uint4* sinv16, int* sexp, hipStream_t s);
// right-hand-side group the autotuner chose for this shape (0 = not tuned yet)
int tuned_group(int es, int bpmax, int nsub, int nrhs, int gnx, int gny);
// The tuned launch of that key: out = {group, waves per item, variant (numbered as the sweep
// policy that forces it), waves per workgroup}; false if not tuned yet.
bool tuned_config(int es, int bpmax, int nsub, int nrhs, int gnx, int gny, int out[4]);
// process-wide sweep policy: 0 autotune over all variants, 1 one-item sweeps,
// 2 the pipelined persistent sweep wherever it fits
void set_sweep_policy(int policy);
int sweep_policy();

// ---- Krylov (ops_krylov.hip) -----------------------------------------------
// blocks of the two-stage reductions (sizes of the partial-sum buffers)
constexpr int RED_BLOCKS = 4096;
void launch_fill(z64* p, long long n, hipStream_t s);  // zero
void launch_copy(const z64* a, z64* b, long long n, hipStream_t s);
void launch_to_node_major(const z64* in, z64* out, long long len, int nrhs, hipStream_t s);
void launch_to_field_major(const z64* in, z64* out, long long len, int nrhs, hipStream_t s);
// out[i][c] = in[i][cols[c]] for c < nout (cols: device array of column indices < nin)
void launch_gather_cols(const z64* in, int nin, const int* cols, int nout, long long len, z64* out, hipStream_t s);
// h[v][r] = sum_node conj(V_v[node][r]) w[node][r], v < nv; V_v = V + v*vstride
void launch_dots(const z64* V, long long vstride, int nv, const z64* w, long long len, int nrhs,
                 z64* partial, z64* h, hipStream_t s, double* npart = nullptr,
                 double* nrm2 = nullptr);
// w -= sum_v h[v][r] V_v ; optionally nrm2[r] = ||w||^2 after the update.  With
// skip given, every kernel of the update returns at once when *skip != 0 (a
// decision taken on the device, so the sequence stays capturable).
void launch_axpy_multi(const z64* V, long long vstride, int nv, const z64* h, z64* w,
                       long long len, int nrhs, double* partial, double* nrm2, hipStream_t s,
                       const int* skip = nullptr);
void launch_norm2(const z64* w, long long len, int nrhs, double* partial, double* nrm2,
                  hipStream_t s);
// w -= sum_v h[v][r] V_v and h2[v][r] = sum_node conj(V_v) w (updated w), one pass;
// false when nv or the batch is too large for the fused kernel
bool launch_axpy_dots(const z64* V, long long vstride, int nv, const z64* h, z64* w, long long len, int nrhs,
                      z64* partial, z64* h2, hipStream_t s, double* npart = nullptr, double* nrm2 = nullptr);
// out[node][r] = fac[r] * w[node][r]
void launch_scale(const z64* w, const double* fac, z64* out, long long len, int nrhs, hipStream_t s);
// x += sum_v y[v][r] Z_v
void launch_update(const z64* Z, long long zstride, int nv, const z64* y, z64* x, long long len,
                   int nrhs, hipStream_t s);
// a = a - b
void launch_sub(z64* a, const z64* b, long long n, hipStream_t s);

// Block Krylov kernels (block FGMRES): block vectors are batches of s <= 32
// right-hand sides, node-major; coefficient blocks [block][32][32] (padded).
// Chunks of the two-stage block reductions for vectors of len nodes.
int block_chunks(long long len);
// C[i] = V_i^H W, i < nv (V_i = V + i * vstride); partial holds
// block_chunks(len) * nv * 1024 elements.  Deterministic.
void launch_block_dots(const z64* V, long long vstride, int nv, const z64* W, long long len, int s, z64* partial,
                       z64* C, hipStream_t st);
// out = (accumulate ? out : 0) + sign sum_{i < nv} In_i C[i]  (In_i = In + i * istride; out aliases no In_i)
void launch_block_gemm(const z64* In, long long istride, int nv, const z64* C, long long len, int s, double sign,
                       bool accumulate, z64* out, hipStream_t st);

// Per-right-hand-side GMRES state (device arrays of length nrhs unless noted).
struct KrylovState {
  int m, nrhs;
  z64* Rm;        // [m+1][m][nrhs] rotated Hessenberg (upper triangle used)
  z64* g;         // [m+1][nrhs]
  double* cs;     // [m][nrhs]
  z64* sn;        // [m][nrhs]
  z64* y;         // [m][nrhs]
  z64* h;         // [m+1][nrhs] coefficients of the current step (h1 + h2)
  z64* h2;        // [m+1][nrhs] second pass
  double* nrm2;   // [nrhs] squared norm of w after orthogonalisation
  double* w0;     // [nrhs] squared norm of w before orthogonalisation
  double* bnorm;  // [nrhs]
  double* beta;   // [nrhs]
  double* est;    // [nrhs]
  double* fac;    // [nrhs] scaling applied to w to form the next basis vector
  int* it;        // [nrhs] total iterations
  int* kc;        // [nrhs] steps in the current cycle
  int* active;    // [nrhs]
  int* done;      // [nrhs]
  int* conv;      // [nrhs] 1 if converged
  int* counter;   // [1] number still active (host reads it)
  double* w1;     // [nrhs] squared norm of w after the first Gram-Schmidt update
  int* skip;      // [1] 1 when the second update of this step is negligible for every RHS
  double* extra;  // [1] algorithmic bytes of the second updates that ran (solve accounting)
};
// Second Gram-Schmidt pass: when sum_v |h2[v][r]|^2 <= tau2 ||w'||^2 for every
// active right-hand side, the second update would change w' by less than
// sqrt(tau2) relative: skip it (h2 := 0, ||w||^2 := ||w'||^2); otherwise let it
// run and add vec_bytes (nv + 2) to *extra.
void launch_reorth_check(KrylovState st, int nv, double tau2, double vec_bytes, hipStream_t s);
void launch_krylov_init(KrylovState st, const double* bn2, hipStream_t s);
// start a cycle from residual norms^2 in beta2: decide done/active, set g[0], fac = 1/beta
void launch_cycle_start(KrylovState st, const double* beta2, double tol, int maxit, int first,
                        hipStream_t s);
void launch_cycle_start_fixed(KrylovState st, const double* beta2, hipStream_t s);
void launch_givens(KrylovState st, int j, double tol, int maxit, int fixed, hipStream_t s);
void launch_backsolve(KrylovState st, hipStream_t s);
void launch_add2(z64* a, const z64* b, long long n, hipStream_t s);
