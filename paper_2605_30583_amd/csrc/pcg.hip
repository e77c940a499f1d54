// Block-Jacobi preconditioned conjugate gradients on the damped normal
// equations (PCGNR, Section V and the paper's glossary): one preconditioner
// block per camera (9x9) and per point (3x3), the diagonal blocks of
// J^T J + lambda D, inverted by Cholesky in float64.
//
// All PCG scalars (rho, alpha, beta, |r|^2, the stop flag) stay on the
// device: every kernel reads them and returns at once when the solve is
// done, so the host enqueues several iterations between polls.  Dot
// products are accumulated in float64 per workgroup and summed in a fixed
// order by a single-workgroup kernel (deterministic).
#include <cmath>

#include "common.hpp"
#include "model.hpp"

namespace cba {

__host__ __device__ constexpr int tri_idx(int n, int k, int l) {
  return k * n - k * (k - 1) / 2 + (l - k);
}

// Cholesky factor L of A + jitter I (lower triangle).  Every loop has a
// fixed trip count, so the matrices stay in registers; a non-positive or
// non-finite pivot makes the result false (the factor is then garbage and
// is not used).
template <int n>
__device__ inline bool cholesky(const double (&A)[n][n], double jitter, double (&L)[n][n]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < n; ++j) {
    double s = A[j][j] + jitter;
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    ok = ok & (s > 0.0) & (bool)isfinite(s);
    L[j][j] = sqrt(s);
#pragma unroll
    for (int i = j + 1; i < n; ++i) {
      double t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  return ok;
}

// Inverse of the n x n symmetric positive definite matrix given by its packed
// upper triangle plus lambda * diag(d); result packed the same way.
// Cholesky A = L L^T, W = L^-1, A^-1 = W^T W.  On a non-positive pivot the
// diagonal is raised by 1e-12 trace(A) and the factorisation retried once;
// if that fails too the inverse of the diagonal is returned.
template <int n>
__device__ void spd_inverse(const double* __restrict__ Hup, const double* dg, double lambda,
                            double* __restrict__ out) {
  double A[n][n], L[n][n], W[n][n];
  double tr = 0.0;
#pragma unroll
  for (int k = 0; k < n; ++k)
#pragma unroll
    for (int l = k; l < n; ++l) {
      const double v = Hup[tri_idx(n, k, l)] + (k == l ? lambda * dg[k] : 0.0);
      A[k][l] = v;
      A[l][k] = v;
      if (k == l) tr += v;
    }
  bool ok = cholesky<n>(A, 0.0, L);
  if (!ok) ok = cholesky<n>(A, 1e-12 * fabs(tr), L);
  if (!ok) {
#pragma unroll
    for (int k = 0; k < n; ++k)
#pragma unroll
      for (int l = k; l < n; ++l) out[tri_idx(n, k, l)] = (k == l && A[k][k] > 0.0) ? 1.0 / A[k][k] : 0.0;
    return;
  }
#pragma unroll
  for (int j = 0; j < n; ++j) {
    W[j][j] = 1.0 / L[j][j];
#pragma unroll
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < i; ++k) s += L[i][k] * W[k][j];
      W[i][j] = -s / L[i][i];
    }
  }
#pragma unroll
  for (int a = 0; a < n; ++a)
#pragma unroll
    for (int b = a; b < n; ++b) {
      double s = 0.0;
#pragma unroll
      for (int m = b; m < n; ++m) s += W[m][a] * W[m][b];
      out[tri_idx(n, a, b)] = s;
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_bj_cams(int nc, const double* __restrict__ Hcc, const S* __restrict__ D,
                                                 double lambda, S* __restrict__ Mc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double dg[9], inv[45];
#pragma unroll
  for (int k = 0; k < 9; ++k) dg[k] = (double)D[9 * (size_t)c + k];
  spd_inverse<9>(Hcc + 45 * (size_t)c, dg, lambda, inv);
#pragma unroll
  for (int k = 0; k < 45; ++k) Mc[45 * (size_t)c + k] = (S)inv[k];
}

template <typename S>
__global__ __launch_bounds__(256) void k_bj_points(int np, const double* __restrict__ Hpp, const S* __restrict__ Dp,
                                                   double lambda, S* __restrict__ Mp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double dg[3], inv[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) dg[k] = (double)Dp[3 * (size_t)i + k];
  spd_inverse<3>(Hpp + 6 * (size_t)i, dg, lambda, inv);
#pragma unroll
  for (int k = 0; k < 6; ++k) Mp[6 * (size_t)i + k] = (S)inv[k];
}

// z = M^-1 r for block b (camera if b < nc, else point b - nc).
template <typename S, int n>
__device__ inline void block_apply(const S* __restrict__ Minv, const S* rv, S* __restrict__ z, double& rz,
                                   double& rr) {
  S mv[n * (n + 1) / 2];
#pragma unroll
  for (int k = 0; k < n * (n + 1) / 2; ++k) mv[k] = Minv[k];
#pragma unroll
  for (int k = 0; k < n; ++k) {
    S s = (S)0;
#pragma unroll
    for (int l = 0; l < n; ++l) s = fma(mv[k <= l ? tri_idx(n, k, l) : tri_idx(n, l, k)], rv[l], s);
    z[k] = s;
    rz = fma((double)rv[k], (double)s, rz);
    rr = fma((double)rv[k], (double)rv[k], rr);
  }
}

template <typename S>
__global__ void k_bj_apply(int nc, int np, const S* __restrict__ Mc, const S* __restrict__ Mp,
                           const S* __restrict__ r, S* __restrict__ z) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (b < nc) {
    block_apply<S, 9>(Mc + 45 * b, r + 9 * b, z + 9 * b, rz, rr);
  } else if (b < (int64_t)nc + np) {
    const int64_t i = b - nc;
    const size_t o = 9 * (size_t)nc + 3 * (size_t)i;
    block_apply<S, 3>(Mp + 6 * i, r + o, z + o, rz, rr);
  }
}

// One block of the start: x = 0, r = +-b, z = M^-1 r, p = z, held in
// registers between the reads and the writes.
template <typename S, int n>
__device__ inline void init_block(const S* __restrict__ Minv, const S* __restrict__ b, double sign, size_t o,
                                  S* __restrict__ x, S* __restrict__ r, S* __restrict__ z, S* __restrict__ p,
                                  double& rz, double& rr) {
  S rv[n], zv[n];
#pragma unroll
  for (int k = 0; k < n; ++k) rv[k] = (S)(sign * (double)b[o + k]);
  block_apply<S, n>(Minv, rv, zv, rz, rr);
#pragma unroll
  for (int k = 0; k < n; ++k) {
    r[o + k] = rv[k];
    x[o + k] = (S)0;
    z[o + k] = zv[k];
    p[o + k] = zv[k];
  }
}

// x = 0, r = +-b, z = M^-1 r, p = z; partials: r^T z, r^T r.
template <typename S>
__global__ __launch_bounds__(256) void k_pcg_init(int nc, int np, const S* __restrict__ Mc,
                                                  const S* __restrict__ Mp, const S* __restrict__ b,
                                                  double sign, S* __restrict__ x, S* __restrict__ r,
                                                  S* __restrict__ z, S* __restrict__ p,
                                                  double* __restrict__ partials) {
  __shared__ double red[4];
  double rz = 0.0, rr = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // camera blocks: nine lanes of one wave each (row k of M^-1 per lane, the
  // whole-block apply's operations in its order), seven blocks to a wave
  const int lane = threadIdx.x & (kWave - 1);
  if (lane < 63) {
    const int64_t n_groups = ((int64_t)nc + 6) / 7;
    const int j = lane / 9, k = lane - 9 * (lane / 9);
    for (int64_t g = i0 / kWave; g < n_groups; g += stride / kWave) {
      const int64_t c = 7 * g + j;
      if (c >= nc) continue;
      const size_t o = 9 * (size_t)c;
      S rv[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) rv[l] = (S)(sign * (double)b[o + l]);
      const S* __restrict__ m = Mc + 45 * c;
      S zk = (S)0;
#pragma unroll
      for (int l = 0; l < 9; ++l) zk = fma(m[k <= l ? tri_idx(9, k, l) : tri_idx(9, l, k)], rv[l], zk);
      S rk = rv[0];
#pragma unroll
      for (int l = 1; l < 9; ++l) rk = l == k ? rv[l] : rk;
      r[o + k] = rk;
      x[o + k] = (S)0;
      z[o + k] = zk;
      p[o + k] = zk;
      rz = fma((double)rk, (double)zk, rz);
      rr = fma((double)rk, (double)rk, rr);
    }
  }
  for (int64_t i = i0; i < np; i += stride)
    init_block<S, 3>(Mp + 6 * i, b, sign, 9 * (size_t)nc + 3 * (size_t)i, x, r, z, p, rz, rr);
  const double a = block_sum(rz, red);
  const double c = block_sum(rr, red);
  if (threadIdx.x == 0) {
    partials[(size_t)blockIdx.x * kPartialWidth] = a;
    partials[(size_t)blockIdx.x * kPartialWidth + 1] = c;
  }
}

__global__ void k_pcg_scalar0(int n, const double* __restrict__ partials, double tol, int max_iter,
                              DevScalars* sc) {
  __shared__ double red[16];
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a += partials[(size_t)i * kPartialWidth];
    c += partials[(size_t)i * kPartialWidth + 1];
  }
  a = block_sum(a, red);
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    sc->rho = a;
    sc->bb = c;
    sc->rr = c;
    sc->tol2 = tol * tol * c;
    sc->iter = 0;
    sc->max_iter = max_iter;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->done = 0;
    sc->reason = PCG_RUNNING;
    sc->last_x = 0;
    sc->ticket = 0;
    if (c == 0.0) {
      sc->done = 1;
      sc->reason = PCG_ZERO_RHS;
    } else if (!isfinite(a) || !isfinite(c) || max_iter <= 0) {
      sc->done = 1;
      sc->reason = max_iter <= 0 ? PCG_MAXITER : PCG_BREAKDOWN;
    }
  }
}

// x += alpha p; r -= alpha w; z = M^-1 r; partials: r^T r, r^T z.
// Stop test and beta after an update, from |r|^2 (a) and r^T z (c).  Any
// stop set here follows a completed update of r, so its x step (applied by
// the direction kernel) is still due: last_x.
__device__ inline void pcg_scalars_after_update(DevScalars* sc, double a, double c) {
  sc->rr = a;
  if (!isfinite(a) || !isfinite(c)) {
    sc->done = 1;
    sc->reason = PCG_BREAKDOWN;
  } else if (a <= sc->tol2) {
    sc->done = 1;
    sc->reason = PCG_CONVERGED;
  } else {
    sc->beta = c / sc->rho;
    sc->rho = c;
    if (sc->iter >= sc->max_iter) {
      sc->done = 1;
      sc->reason = PCG_MAXITER;
    }
  }
  sc->last_x = sc->done;
}

// r -= alpha w, z = M^-1 r, and the sums r^T r, r^T z.  A camera block
// takes nine lanes of one wave, seven blocks to a wave (lane 9 j + k: row k
// of block j): each lane recomputes the block's nine updated r values and
// applies row k of M^-1 (the same operations, in the same order, as the
// whole-block apply), so a 9x9 block does not serialise one thread on 45
// loads and 81 multiply-adds, which on a small problem is the kernel's
// critical path.  The nine lanes of a block are in one wave, so all of them
// read r before any writes it.  Thread i also takes point block i
// (grid-stride, its r and w in registers).  Workgroup sums go to the partial
// slots.  The x step of the same iteration is taken by the direction kernel,
// which reads p anyway.
//
// LAST (a small problem, few workgroups): instead of a separate launch of
// k_pcg_scalar1, the last workgroup to finish sums the partials and sets the
// scalars.  Each workgroup takes a ticket with a device-scope release (its
// partials, written by the same thread, become visible first); the thread
// that takes the last ticket acquires every workgroup's partials with a
// device-scope acquire fence after its ticket read, and the workgroup barrier
// passes them on to its other threads.  The release writes back the L2 of the
// workgroup's XCD, which on a large problem (megabytes of r and z in flight)
// costs more than the launch it saves.
template <typename S, bool LAST>
__global__ __launch_bounds__(256) void k_pcg_update(int nc, int np, const S* __restrict__ Mc,
                                                    const S* __restrict__ Mp, S* __restrict__ r,
                                                    S* __restrict__ z, const S* __restrict__ w,
                                                    DevScalars* __restrict__ sc,
                                                    double* __restrict__ partials) {
  __shared__ double red[4];
  if (sc->done) return;
  const double alpha = sc->alpha;
  double rz = 0.0, rr = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  if (lane < 63) {
    const int64_t n_groups = ((int64_t)nc + 6) / 7;
    const int j = lane / 9, k = lane - 9 * (lane / 9);
    for (int64_t g = i0 / kWave; g < n_groups; g += stride / kWave) {
      const int64_t c = 7 * g + j;
      if (c >= nc) continue;
      const size_t o = 9 * (size_t)c;
      S rv[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) rv[l] = (S)fma(-alpha, (double)w[o + l], (double)r[o + l]);
      const S* __restrict__ m = Mc + 45 * c;
      S zk = (S)0;
#pragma unroll
      for (int l = 0; l < 9; ++l) zk = fma(m[k <= l ? tri_idx(9, k, l) : tri_idx(9, l, k)], rv[l], zk);
      S rk = rv[0];
#pragma unroll
      for (int l = 1; l < 9; ++l) rk = l == k ? rv[l] : rk;
      r[o + k] = rk;
      z[o + k] = zk;
      rz = fma((double)rk, (double)zk, rz);
      rr = fma((double)rk, (double)rk, rr);
    }
  }
  const S* __restrict__ wp = w + 9 * (size_t)nc;
  S* __restrict__ rp = r + 9 * (size_t)nc;
  S* __restrict__ zp = z + 9 * (size_t)nc;
  for (int64_t i = i0; i < np; i += stride) {
    const size_t o = 3 * (size_t)i;
    S wv[3], rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      wv[k] = wp[o + k];
      rv[k] = rp[o + k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      rv[k] = (S)fma(-alpha, (double)wv[k], (double)rv[k]);
      rp[o + k] = rv[k];
    }
    block_apply<S, 3>(Mp + 6 * i, rv, zp + o, rz, rr);
  }
  const double sa = block_sum(rr, red);
  const double sz = block_sum(rz, red);
  if (threadIdx.x == 0) {
    partials[(size_t)blockIdx.x * kPartialWidth] = sa;
    partials[(size_t)blockIdx.x * kPartialWidth + 1] = sz;
  }
  if constexpr (LAST) {
    __shared__ int last;
    if (threadIdx.x == 0) {
      // release this workgroup's partials (written by this thread) with the
      // ticket: a write-back of the XCD's L2, no invalidate
      last = __hip_atomic_fetch_add(&sc->ticket, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) ==
             gridDim.x - 1;
      // the last ticket's holder acquires every workgroup's partials: its
      // ticket read is the atomic this fence pairs with (only the last
      // workgroup invalidates its caches); the barrier below passes them on
      // to the workgroup's other threads
      if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (last) {
      double a = 0.0, c = 0.0;
      for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) {
        a += partials[(size_t)i * kPartialWidth];
        c += partials[(size_t)i * kPartialWidth + 1];
      }
      a = block_sum(a, red);
      c = block_sum(c, red);
      if (threadIdx.x == 0) {
        pcg_scalars_after_update(sc, a, c);
        sc->ticket = 0;
      }
    }
  }
}

// Sums the update's partials in slot order (deterministic) and sets the PCG
// scalars.  A separate single-workgroup launch on a large problem: folding
// this into the update's last workgroup (as the small-problem variant does)
// needs a device-scope fence per workgroup, which writes back the L2 of its
// XCD and there costs more than the launch.
__global__ void k_pcg_scalar1(int n, const double* __restrict__ partials, DevScalars* sc) {
  __shared__ double red[16];
  if (sc->done) return;
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a += partials[(size_t)i * kPartialWidth];
    c += partials[(size_t)i * kPartialWidth + 1];
  }
  a = block_sum(a, red);
  c = block_sum(c, red);
  if (threadIdx.x == 0) pcg_scalars_after_update(sc, a, c);
}

// The iteration's x step x += alpha p with the current p, then the new
// direction p = z + beta p unless the iteration stopped the solve; four
// elements per thread with 16-byte vector accesses.  The camera part of p
// is also written to the camera rows that the next product gathers from.
// A solve stopped by an earlier iteration (or by the product's breakdown
// test, before any update) leaves x alone.
template <typename S>
__global__ __launch_bounds__(256) void k_pcg_p(int64_t N, int nc, const S* __restrict__ z, S* __restrict__ p,
                                               S* __restrict__ x, S* __restrict__ p_cam, int row_stride,
                                               int row_off, const DevScalars* __restrict__ sc) {
  using V = S __attribute__((ext_vector_type(4)));
  if (sc->done && !sc->last_x) return;
  const bool new_dir = !sc->done;
  const double alpha = sc->alpha;
  const double beta = sc->beta;
  const int64_t ncam = 9 * (int64_t)nc;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  auto to_row = [&](int64_t e, S v) {
    if (e < ncam) p_cam[(e / 9) * row_stride + row_off + e % 9] = v;
  };
  const int64_t n4 = N / 4;
  const V* __restrict__ z4 = reinterpret_cast<const V*>(z);
  V* __restrict__ p4 = reinterpret_cast<V*>(p);
  V* __restrict__ x4 = reinterpret_cast<V*>(x);
  for (int64_t q = i0; q < n4; q += stride) {
    const V pv = p4[q];
    const V xv = x4[q];
    V xo;
#pragma unroll
    for (int k = 0; k < 4; ++k) xo[k] = (S)fma(alpha, (double)pv[k], (double)xv[k]);
    x4[q] = xo;
    if (new_dir) {
      const V zv = z4[q];
      V o;
#pragma unroll
      for (int k = 0; k < 4; ++k) o[k] = (S)fma(beta, (double)pv[k], (double)zv[k]);
      p4[q] = o;
      if (4 * q < ncam) {
#pragma unroll
        for (int k = 0; k < 4; ++k) to_row(4 * q + k, o[k]);
      }
    }
  }
  for (int64_t e = 4 * n4 + i0; e < N; e += stride) {
    const S pe = p[e];
    x[e] = (S)fma(alpha, (double)pe, (double)x[e]);
    if (new_dir) {
      const S o = (S)fma(beta, (double)pe, (double)z[e]);
      p[e] = o;
      to_row(e, o);
    }
  }
}

// Partials of sum a b and (if e) sum a e b.
template <typename S>
__global__ __launch_bounds__(256) void k_dot(int64_t N, const S* __restrict__ a, const S* __restrict__ b,
                                             const S* __restrict__ e, double* __restrict__ partials) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double t = (double)a[i] * (double)b[i];
    s = e ? fma(t, (double)e[i], s) : s + t;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kPartialWidth] = s;
}

// Partials of the three sums of the LM predicted decrease: g^T x, x^T r and
// x^T D x, in one pass.
template <typename S>
__global__ __launch_bounds__(256) void k_pred_dots(int64_t N, const S* __restrict__ g, const S* __restrict__ x,
                                                   const S* __restrict__ r, const S* __restrict__ D,
                                                   double* __restrict__ partials) {
  __shared__ double red[4];
  double gx = 0.0, xr = 0.0, xdx = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const double xv = x[i];
    gx = fma((double)g[i], xv, gx);
    xr = fma(xv, (double)r[i], xr);
    xdx = fma(xv * xv, (double)D[i], xdx);
  }
  gx = block_sum(gx, red);
  xr = block_sum(xr, red);
  xdx = block_sum(xdx, red);
  if (threadIdx.x == 0) {
    partials[(size_t)blockIdx.x * kPartialWidth] = gx;
    partials[(size_t)blockIdx.x * kPartialWidth + 1] = xr;
    partials[(size_t)blockIdx.x * kPartialWidth + 2] = xdx;
  }
}

__global__ void k_reduce_pred(int n, const double* __restrict__ partials, DevScalars* sc) {
  __shared__ double red[16];
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x)
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] += partials[(size_t)i * kPartialWidth + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = block_sum(v[k], red);
    if (threadIdx.x == 0) sc->red[4 + k] = t;
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_absmax(int64_t N, const S* __restrict__ a, double* __restrict__ partials) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    s = fmax(s, fabs((double)a[i]));
  s = block_max(s, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kPartialWidth] = s;
}

__global__ void k_reduce_partials(int n, const double* __restrict__ partials, int is_max, DevScalars* sc,
                                  int slot) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = partials[(size_t)i * kPartialWidth];
    s = is_max ? fmax(s, v) : s + v;
  }
  s = is_max ? block_max(s, red) : block_sum(s, red);
  if (threadIdx.x == 0) sc->red[slot] = s;
}

template <typename S>
__global__ void k_vec_to_caller(int nc, int np, const int* __restrict__ cam_c2i, const int* __restrict__ pt_c2i,
                                const S* __restrict__ in, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ncam = 9 * (int64_t)nc;
  if (i < ncam) {
    out[i] = (double)in[9 * (size_t)cam_c2i[i / 9] + i % 9];
  } else if (i < ncam + 3 * (int64_t)np) {
    const int64_t j = i - ncam;
    out[i] = (double)in[ncam + 3 * (size_t)pt_c2i[j / 3] + j % 3];
  }
}

template <typename S>
__global__ void k_vec_from_caller(int nc, int np, const int* __restrict__ cam_c2i, const int* __restrict__ pt_c2i,
                                  const double* __restrict__ in, S* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ncam = 9 * (int64_t)nc;
  if (i < ncam) {
    out[9 * (size_t)cam_c2i[i / 9] + i % 9] = (S)in[i];
  } else if (i < ncam + 3 * (int64_t)np) {
    const int64_t j = i - ncam;
    out[ncam + 3 * (size_t)pt_c2i[j / 3] + j % 3] = (S)in[i];
  }
}

// ---------------------------------------------------------------------------
// Host drivers.
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int threads) {
  return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads);
}

static inline unsigned vec_grid(int64_t n) { return (unsigned)std::min<int64_t>(nblk(n, 256), 1024); }

template <typename S>
static void block_jacobi_t(caspar_ba* h, double lambda) {
  hipStream_t st = h->stream;
  if (h->nc) {
    k_bj_cams<S><<<nblk(h->nc, 64), 64, 0, st>>>(h->nc, h->Hcc, (const S*)h->vec.D, lambda, (S*)h->Mc);
    CBA_LAUNCHED();
  }
  if (h->np) {
    k_bj_points<S><<<nblk(h->np, 256), 256, 0, st>>>(h->np, h->Hpp, (const S*)h->vec.D + 9 * (size_t)h->nc,
                                                     lambda, (S*)h->Mp);
    CBA_LAUNCHED();
  }
}

void run_block_jacobi(caspar_ba* h, double lambda) {
  if (h->bj_lambda == lambda) return;
  if (h->prec == CASPAR_FP64)
    block_jacobi_t<double>(h, lambda);
  else
    block_jacobi_t<float>(h, lambda);
  h->bj_lambda = lambda;
}

void run_bj_apply(caspar_ba* h, const void* r, void* z) {
  const int64_t nb = (int64_t)h->nc + h->np;
  if (nb == 0) return;
  if (h->prec == CASPAR_FP64)
    k_bj_apply<double><<<nblk(nb, 256), 256, 0, h->stream>>>(h->nc, h->np, (const double*)h->Mc,
                                                             (const double*)h->Mp, (const double*)r, (double*)z);
  else
    k_bj_apply<float><<<nblk(nb, 256), 256, 0, h->stream>>>(h->nc, h->np, (const float*)h->Mc,
                                                            (const float*)h->Mp, (const float*)r, (float*)z);
  CBA_LAUNCHED();
}

// The update sets the PCG scalars itself (no k_pcg_scalar1 launch) up to
// this many workgroups (points or cameras up to 256 per workgroup).
constexpr unsigned kLastGroupMaxGroups = 256;

template <typename S>
static int pcg_t(caspar_ba* h, double lambda, const S* b, bool negate, double tol, int max_iters,
                 int check_every, double* rel_resid, int first_batch) {
  hipStream_t st = h->stream;
  const int64_t nb = (int64_t)h->nc + h->np;
  const int64_t N = h->N;
  S* x = (S*)h->vec.x;
  S* r = (S*)h->vec.r;
  S* z = (S*)h->vec.z;
  S* p = (S*)h->vec.p;
  S* w = (S*)h->vec.w;
  const S* Mc = (const S*)h->Mc;
  const S* Mp = (const S*)h->Mp;
  run_block_jacobi(h, lambda);
  const unsigned vg = vec_grid(std::max<int64_t>(nb, 1));
  k_pcg_init<S><<<vg, 256, 0, st>>>(h->nc, h->np, Mc, Mp, b, negate ? -1.0 : 1.0, x, r, z, p, h->partials);
  CBA_LAUNCHED();
  k_pcg_scalar0<<<1, 1024, 0, st>>>((int)vg, h->partials, tol, max_iters, h->scal);
  CBA_LAUNCHED();
  const unsigned ug = (unsigned)std::min<int64_t>(nblk(std::max<int64_t>(std::max(h->nc, h->np), 1), 256),
                                                  kMaxPartials);
  const unsigned pg = (unsigned)std::min<int64_t>(nblk(std::max<int64_t>(N / 4, 1), 256), 4096);
  check_every = std::max(1, check_every);
  // the first batch is enqueued without reading the start state: if the
  // start already stopped PCG (zero right-hand side, no iterations allowed),
  // its kernels exit at once.  The caller may size it from an expected
  // iteration count (successive LM steps need similar counts), so the host
  // reads back about twice per solve instead of every check_every.
  DevScalars s{};
  int launched = 0;
  int batch = std::max(check_every, std::min(first_batch, max_iters));
  do {
    for (int k = 0; k < batch; ++k) {
      // the first product pads the camera rows of p itself; later ones use
      // the rows written by k_pcg_p
      run_matvec(h, lambda, p, w, true, launched + k == 0);
      if (ug <= kLastGroupMaxGroups) {
        k_pcg_update<S, true><<<ug, 256, 0, st>>>(h->nc, h->np, Mc, Mp, r, z, w, h->scal, h->partials);
        CBA_LAUNCHED();
      } else {
        k_pcg_update<S, false><<<ug, 256, 0, st>>>(h->nc, h->np, Mc, Mp, r, z, w, h->scal, h->partials);
        CBA_LAUNCHED();
        k_pcg_scalar1<<<1, 1024, 0, st>>>((int)ug, h->partials, h->scal);
        CBA_LAUNCHED();
      }
      k_pcg_p<S><<<pg, 256, 0, st>>>(N, h->nc, z, p, x, (S*)h->p_cam, cam_row_stride<S>(h), cam_row_p_off(h),
                                     h->scal);
      CBA_LAUNCHED();
    }
    launched += batch;
    batch = check_every;
    s = read_scalars(h);
  } while (!s.done && launched <= max_iters);
  timing_harvest(h, s.iter);
  if (!s.done) fail(CASPAR_ENUMERIC, "internal: PCG did not reach its stop condition");
  if (rel_resid) *rel_resid = s.bb > 0.0 ? std::sqrt(std::max(s.rr, 0.0) / s.bb) : 0.0;
  return s.iter;
}

int run_pcg(caspar_ba* h, double lambda, const void* b, bool negate_b, double tol, int max_iters,
            int check_every, void* x, double* rel_resid, int first_batch) {
  (void)x;
  if (h->prec == CASPAR_FP64)
    return pcg_t<double>(h, lambda, (const double*)b, negate_b, tol, max_iters, check_every, rel_resid,
                         first_batch);
  return pcg_t<float>(h, lambda, (const float*)b, negate_b, tol, max_iters, check_every, rel_resid, first_batch);
}

void launch_pred_dots(caspar_ba* h) {
  const int64_t N = h->N;
  if (N == 0) return;
  const unsigned g = vec_grid(N);
  if (h->prec == CASPAR_FP64)
    k_pred_dots<double><<<g, 256, 0, h->stream>>>(N, (const double*)h->vec.g, (const double*)h->vec.x,
                                                  (const double*)h->vec.r, (const double*)h->vec.D, h->partials);
  else
    k_pred_dots<float><<<g, 256, 0, h->stream>>>(N, (const float*)h->vec.g, (const float*)h->vec.x,
                                                 (const float*)h->vec.r, (const float*)h->vec.D, h->partials);
  CBA_LAUNCHED();
  k_reduce_pred<<<1, 1024, 0, h->stream>>>((int)g, h->partials, h->scal);
  CBA_LAUNCHED();
}

void pred_dots_of(const caspar_ba* h, const DevScalars& sc, double* gx, double* xr, double* xDx) {
  const bool any = h->N > 0;
  *gx = any ? sc.red[4] : 0.0;
  *xr = any ? sc.red[5] : 0.0;
  *xDx = any ? sc.red[6] : 0.0;
}

void run_pred_dots(caspar_ba* h, double* gx, double* xr, double* xDx) {
  launch_pred_dots(h);
  pred_dots_of(h, read_scalars(h), gx, xr, xDx);
}

double run_dot(caspar_ba* h, const void* a, const void* b, const void* e) {
  const int64_t N = h->N;
  if (N == 0) return 0.0;
  const unsigned g = vec_grid(N);
  if (h->prec == CASPAR_FP64)
    k_dot<double><<<g, 256, 0, h->stream>>>(N, (const double*)a, (const double*)b, (const double*)e, h->partials);
  else
    k_dot<float><<<g, 256, 0, h->stream>>>(N, (const float*)a, (const float*)b, (const float*)e, h->partials);
  CBA_LAUNCHED();
  k_reduce_partials<<<1, 1024, 0, h->stream>>>((int)g, h->partials, 0, h->scal, 2);
  CBA_LAUNCHED();
  return read_scalars(h).red[2];
}

void launch_absmax(caspar_ba* h, const void* a) {
  const int64_t N = h->N;
  if (N == 0) return;
  const unsigned g = vec_grid(N);
  if (h->prec == CASPAR_FP64)
    k_absmax<double><<<g, 256, 0, h->stream>>>(N, (const double*)a, h->partials);
  else
    k_absmax<float><<<g, 256, 0, h->stream>>>(N, (const float*)a, h->partials);
  CBA_LAUNCHED();
  k_reduce_partials<<<1, 1024, 0, h->stream>>>((int)g, h->partials, 1, h->scal, 3);
  CBA_LAUNCHED();
}

double run_absmax(caspar_ba* h, const void* a) {
  if (h->N == 0) return 0.0;
  launch_absmax(h, a);
  return read_scalars(h).red[3];
}

void run_to_caller_vector(caspar_ba* h, const void* in, double* out) {
  const int64_t N = h->N;
  if (N == 0) return;
  if (h->prec == CASPAR_FP64)
    k_vec_to_caller<double><<<nblk(N, 256), 256, 0, h->stream>>>(h->nc, h->np, h->cam_c2i, h->pt_c2i,
                                                                 (const double*)in, out);
  else
    k_vec_to_caller<float><<<nblk(N, 256), 256, 0, h->stream>>>(h->nc, h->np, h->cam_c2i, h->pt_c2i,
                                                                (const float*)in, out);
  CBA_LAUNCHED();
}

void run_from_caller_vector(caspar_ba* h, const double* in, void* out) {
  const int64_t N = h->N;
  if (N == 0) return;
  if (h->prec == CASPAR_FP64)
    k_vec_from_caller<double><<<nblk(N, 256), 256, 0, h->stream>>>(h->nc, h->np, h->cam_c2i, h->pt_c2i, in,
                                                                   (double*)out);
  else
    k_vec_from_caller<float><<<nblk(N, 256), 256, 0, h->stream>>>(h->nc, h->np, h->cam_c2i, h->pt_c2i, in,
                                                                  (float*)out);
  CBA_LAUNCHED();
}

void run_zero(caspar_ba* h, void* v, size_t count) {
  if (count) CBA_HIP(hipMemsetAsync(v, 0, count * scalar_bytes(h->prec), h->stream));
}

}  // namespace cba
