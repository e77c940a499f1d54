// Levenberg-Marquardt driver (Section V: gain-ratio damping update after
// Madsen et al., tangent-space retraction, normal equations solved by
// block-Jacobi PCG without a Schur reduction), the parity hooks and the
// implicit adjoint of the optimum.
//
// One LM iteration:
//   solve (J^T J + lambda D) delta = -g by PCG
//   pred = 1/2 (b^T delta + delta^T r_pcg + lambda delta^T D delta), b = -g
//   rho  = (F - F(theta (+) delta)) / pred
//   rho > 0 and pred > 0: accept, relinearise,
//                         lambda *= max(1/3, 1 - (2 rho - 1)^3), nu = 2
//   otherwise:            lambda *= nu, nu *= 2
//   lambda clamped to [lambda_min, lambda_max].
#include <chrono>
#include <cmath>
#include <limits>

#include "common.hpp"
#include "model.hpp"

namespace cba {

// Right-hand side of the adjoint: caller gradients -> internal tangent order.
// Cameras: d/d(angle-axis) -> d/d(right perturbation) with J_r^-1(w)^T.
template <typename S>
__global__ void k_adjoint_rhs(int nc, int np, const double* __restrict__ cam, const int* __restrict__ cam_c2i,
                              const int* __restrict__ pt_c2i, const double* __restrict__ gc,
                              const double* __restrict__ gp, S* __restrict__ v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nc) {
    const int ci = cam_c2i[i];
    S* o = v + 9 * (size_t)ci;
    if (!gc) {
      for (int k = 0; k < 9; ++k) o[k] = (S)0;
      return;
    }
    const double* g = gc + 9 * (size_t)i;
    const double* row = cam + (size_t)ci * kCamStride;
    double R[9], w[3], t[3];
    for (int k = 0; k < 9; ++k) R[k] = row[k];
    so3_log(R, w);
    so3_grad_to_tangent(w, g, t);
    for (int k = 0; k < 3; ++k) o[k] = (S)t[k];
    for (int k = 3; k < 9; ++k) o[k] = (S)g[k];
  } else if (i < (int64_t)nc + np) {
    const int64_t p = i - nc;
    S* o = v + 9 * (size_t)nc + 3 * (size_t)pt_c2i[p];
    for (int k = 0; k < 3; ++k) o[k] = gp ? (S)gp[3 * p + k] : (S)0;
  }
}

// Gauge directions at the current parameters, right-perturbation tangent:
//   rotation about e_k:    dw = -e_k,            dX = e_k x X
//   translation along e_k: dt = -R e_k,          dX = e_k
//   scale:                 dt = t,               dX = X
// n[a][i] for the block's components (9 for a camera, 3 for a point).
__device__ inline void gauge_block(bool cam, const double* row_or_X, double n[7][9]) {
  for (int a = 0; a < 7; ++a)
    for (int i = 0; i < 9; ++i) n[a][i] = 0.0;
  if (cam) {
    const double* R = row_or_X;
    const double* t = row_or_X + 9;
    for (int k = 0; k < 3; ++k) {
      n[k][k] = -1.0;
      for (int j = 0; j < 3; ++j) n[3 + k][3 + j] = -R[3 * j + k];
    }
    for (int j = 0; j < 3; ++j) n[6][3 + j] = t[j];
  } else {
    const double* X = row_or_X;
    n[0][0] = 0.0;  n[0][1] = -X[2]; n[0][2] = X[1];   // e_0 x X
    n[1][0] = X[2]; n[1][1] = 0.0;   n[1][2] = -X[0];  // e_1 x X
    n[2][0] = -X[1]; n[2][1] = X[0]; n[2][2] = 0.0;    // e_2 x X
    for (int k = 0; k < 3; ++k) n[3 + k][k] = 1.0;
    for (int j = 0; j < 3; ++j) n[6][j] = X[j];
  }
}

constexpr int kGaugeStats = 35;  // 28 entries of N^T D N (upper) + 7 of N^T g

template <typename S>
__global__ __launch_bounds__(256) void k_gauge_stats(int nc, int np, const double* __restrict__ cam,
                                                     const double* __restrict__ X, const S* __restrict__ D,
                                                     const S* __restrict__ g, double* __restrict__ rows) {
  __shared__ double red[4];
  double acc[kGaugeStats];
  for (int k = 0; k < kGaugeStats; ++k) acc[k] = 0.0;
  const int64_t nb = (int64_t)nc + np;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
    const bool is_cam = b < nc;
    double n[7][9];
    gauge_block(is_cam, is_cam ? cam + (size_t)b * kCamStride : X + 3 * (size_t)(b - nc), n);
    const int len = is_cam ? 9 : 3;
    const size_t o = is_cam ? 9 * (size_t)b : 9 * (size_t)nc + 3 * (size_t)(b - nc);
    for (int i = 0; i < len; ++i) {
      const double d = (double)D[o + i], gi = (double)g[o + i];
      int q = 0;
      for (int a2 = 0; a2 < 7; ++a2)
        for (int c2 = a2; c2 < 7; ++c2) acc[q++] += n[a2][i] * d * n[c2][i];
      for (int a2 = 0; a2 < 7; ++a2) acc[28 + a2] += n[a2][i] * gi;
    }
  }
  for (int k = 0; k < kGaugeStats; ++k) {
    const double s = block_sum(acc[k], red);
    if (threadIdx.x == 0) rows[(size_t)blockIdx.x * kGaugeStats + k] = s;
  }
}

template <typename S>
__global__ void k_gauge_apply(int nc, int np, const double* __restrict__ cam, const double* __restrict__ X,
                              const S* __restrict__ D, S* __restrict__ g, double c0, double c1, double c2, double c3,
                              double c4, double c5, double c6) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= (int64_t)nc + np) return;
  const double c[7] = {c0, c1, c2, c3, c4, c5, c6};
  const bool is_cam = b < nc;
  double n[7][9];
  gauge_block(is_cam, is_cam ? cam + (size_t)b * kCamStride : X + 3 * (size_t)(b - nc), n);
  const int len = is_cam ? 9 : 3;
  const size_t o = is_cam ? 9 * (size_t)b : 9 * (size_t)nc + 3 * (size_t)(b - nc);
  for (int i = 0; i < len; ++i) {
    double s = 0.0;
    for (int a = 0; a < 7; ++a) s += n[a][i] * c[a];
    g[o + i] = (S)((double)g[o + i] - (double)D[o + i] * s);
  }
}

// dL/dpx_o = J_o v in caller order.
template <typename S, bool RJ>
__global__ void k_adjoint_obs(int n_tiles, const Tile* __restrict__ tiles, const uint32_t* __restrict__ meta,
                              const void* __restrict__ J, const S* __restrict__ cam_s,
                              const double* __restrict__ X, const S* __restrict__ v, int nc,
                              const int* __restrict__ s2c, const S* __restrict__ wts, double* __restrict__ out) {
  const int t = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (t >= n_tiles) return;
  const Tile tl = tiles[t];
  if (lane >= tile_nobs(tl.info)) return;
  const int o = tl.obs_begin + lane;
  const uint32_t m = meta[o];
  const int ci = (int)(m & ((1u << kCamBits) - 1));
  const int pi = tl.pt_begin + (int)(m >> kCamBits);
  S col[12][2];
  jacobian_of<S, RJ>(J, cam_s, X, o, ci, pi, col);
  double q0 = 0.0, q1 = 0.0;
  for (int k = 0; k < 9; ++k) {
    const double x = v[9 * (size_t)ci + k];
    q0 = fma((double)col[k][0], x, q0);
    q1 = fma((double)col[k][1], x, q1);
  }
  for (int k = 0; k < 3; ++k) {
    const double x = v[9 * (size_t)nc + 3 * (size_t)pi + k];
    q0 = fma((double)col[9 + k][0], x, q0);
    q1 = fma((double)col[9 + k][1], x, q1);
  }
  // robust loss (weights held fixed): dL/dpx_o = w_o J_o v; stored blocks
  // are sqrt(w)-scaled, recomputed ones are not
  if (wts) {
    const double f = RJ ? (double)wts[o] : sqrt((double)wts[o]);
    q0 *= f;
    q1 *= f;
  }
  const size_t c = (size_t)s2c[o];
  out[2 * c] = q0;
  out[2 * c + 1] = q1;
}

static inline unsigned nblk(int64_t n, int threads) {
  return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads);
}

static void ensure_linearized(caspar_ba* h) {
  if (!h->linearized) run_linearize(h);
}

static void check_device(caspar_ba* h) {
  int dev = -1;
  CBA_HIP(hipGetDevice(&dev));
  if (dev != h->device) CBA_HIP(hipSetDevice(h->device));
}

static void solve_impl(caspar_ba* h, const caspar_solve_opts* opts_in, caspar_solve_stats* stats,
                       caspar_iter_record* hist) {
  caspar_solve_opts o;
  caspar_default_solve_opts(&o);
  if (opts_in) o = *opts_in;
  CBA_REQUIRE(o.max_lm_iters >= 0 && o.max_pcg_iters >= 0, "negative iteration limit");
  CBA_REQUIRE(o.lambda0 > 0.0 && o.lambda_min > 0.0 && o.lambda_max >= o.lambda_min, "bad damping options");
  CBA_REQUIRE(o.pcg_tol >= 0.0, "bad PCG tolerance");
  CBA_REQUIRE(o.pred_tol >= 0.0, "bad predicted-decrease tolerance");
  const auto t_start = std::chrono::steady_clock::now();
  ensure_linearized(h);
  if (!std::isfinite(h->cost)) fail(CASPAR_ENUMERIC, "initial cost is not finite");
  const double F0 = h->cost;
  const double g0 = h->gmax;
  double lam = std::min(std::max(o.lambda0, o.lambda_min), o.lambda_max);
  double nu = 2.0;
  int iters = 0, accepted = 0, pcg_total = 0, reason = 0, prev_pcg = 0;
  for (int it = 0; it < o.max_lm_iters; ++it) {
    if (h->gmax <= o.grad_tol * std::max(1.0, g0)) {
      reason = 1;
      break;
    }
    if (h->cost <= o.min_cost) {
      reason = 2;
      break;
    }
    double rel = 0.0;
    // the previous step's PCG count sizes the first batch before a poll
    const int k = run_pcg(h, lam, h->vec.g, true, o.pcg_tol, o.max_pcg_iters, o.pcg_check_every, nullptr, &rel,
                          prev_pcg - o.pcg_check_every);
    prev_pcg = k;
    pcg_total += k;
    // pred = 1/2 (-g^T x + x^T r + lambda x^T D x); its dot products, the
    // trial parameters and the trial cost are enqueued together and read
    // back once
    launch_pred_dots(h);
    run_retract(h, h->vec.x);
    launch_cost(h, h->cam_trial, h->X_trial, false);
    const DevScalars sc = read_scalars(h);
    double gx, xr, xDx;
    pred_dots_of(h, sc, &gx, &xr, &xDx);
    const double pred = 0.5 * (-gx + xr + lam * xDx);
    if (o.pred_tol > 0.0 && pred <= o.pred_tol * h->cost) {
      // the model predicts no decrease the cost could resolve
      reason = 3;
      break;
    }
    const double Ft = cost_of(h, sc);
    const double F = h->cost;
    const double rho = (pred > 0.0 && std::isfinite(Ft)) ? (F - Ft) / pred
                                                         : -std::numeric_limits<double>::infinity();
    const double lam_used = lam;
    const bool acc = rho > 0.0;
    if (acc) {
      std::swap(h->cam, h->cam_trial);
      std::swap(h->X, h->X_trial);
      h->linearized = false;
      run_linearize(h);
      // the cost of the new parameters is the trial cost the step was
      // accepted on (the linearisation's own sum differs in rounding order),
      // so accepted costs decrease exactly and the next gain ratio compares
      // like with like
      h->cost = Ft;
      lam *= std::max(1.0 / 3.0, 1.0 - std::pow(2.0 * rho - 1.0, 3));
      nu = 2.0;
      ++accepted;
    } else {
      lam *= nu;
      nu = std::min(2.0 * nu, 1152921504606846976.0);  // 2^60
    }
    lam = std::min(std::max(lam, o.lambda_min), o.lambda_max);
    if (hist) {
      caspar_iter_record& r = hist[it];
      r.cost = h->cost;
      r.trial_cost = Ft;
      r.lambda = lam_used;
      r.rho = rho;
      r.pred = pred;
      r.pcg_rel_resid = rel;
      r.accepted = acc ? 1 : 0;
      r.pcg_iters = k;
      r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    }
    ++iters;
  }
  if (stats) {
    stats->lm_iters = iters;
    stats->accepted = accepted;
    stats->pcg_iters_total = pcg_total;
    stats->stop_reason = reason;
    stats->initial_cost = F0;
    stats->final_cost = h->cost;
    stats->final_lambda = lam;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
}

template <typename S>
static void adjoint_rhs_t(caspar_ba* h, const double* gc, const double* gp) {
  const int64_t n = (int64_t)h->nc + h->np;
  if (n == 0) return;
  k_adjoint_rhs<S><<<nblk(n, 256), 256, 0, h->stream>>>(h->nc, h->np, h->cam, h->cam_c2i, h->pt_c2i, gc, gp,
                                                         (S*)h->vec.v);
  CBA_LAUNCHED();
}

template <typename S>
static void adjoint_obs_t(caspar_ba* h, double* out) {
  if (h->n_tiles == 0) return;
  const unsigned grid = nblk((int64_t)h->n_tiles * kWave, 256);
  if (h->rj)
    k_adjoint_obs<S, true><<<grid, 256, 0, h->stream>>>(h->n_tiles, h->tiles, h->meta, h->J, (const S*)h->cam_s,
                                                        h->X, (const S*)h->vec.x, h->nc, h->obs_s2c,
                                                        weights_of<S>(h), out);
  else
    k_adjoint_obs<S, false><<<grid, 256, 0, h->stream>>>(h->n_tiles, h->tiles, h->meta, h->J, (const S*)h->cam_s,
                                                         h->X, (const S*)h->vec.x, h->nc, h->obs_s2c,
                                                        weights_of<S>(h), out);
  CBA_LAUNCHED();
}

// g <- g - D N (N^T D N)^-1 N^T g on the handle's vector v.
template <typename S>
static void gauge_project_t(caspar_ba* h) {
  const int64_t nb = (int64_t)h->nc + h->np;
  if (nb == 0) return;
  const int grid = (int)std::min<int64_t>(256, (nb + 255) / 256);
  k_gauge_stats<S><<<grid, 256, 0, h->stream>>>(h->nc, h->np, h->cam, h->X, (const S*)h->vec.D,
                                                 (const S*)h->vec.v, h->gauge_rows);
  CBA_LAUNCHED();
  std::vector<double> rows((size_t)grid * kGaugeStats);
  CBA_HIP(hipMemcpyAsync(rows.data(), h->gauge_rows, rows.size() * 8, hipMemcpyDeviceToHost, h->stream));
  sync(h);
  double M[7][7], r[7];
  for (int a = 0; a < 7; ++a) r[a] = 0.0;
  for (int a = 0; a < 7; ++a)
    for (int b = 0; b < 7; ++b) M[a][b] = 0.0;
  for (int k = 0; k < grid; ++k) {
    int q = 0;
    for (int a = 0; a < 7; ++a)
      for (int b = a; b < 7; ++b) M[a][b] += rows[(size_t)k * kGaugeStats + q++];
    for (int a = 0; a < 7; ++a) r[a] += rows[(size_t)k * kGaugeStats + 28 + a];
  }
  for (int a = 0; a < 7; ++a)
    for (int b = 0; b < a; ++b) M[a][b] = M[b][a];
  // Gaussian elimination with partial pivoting on the 7x7 system M c = r
  int piv[7];
  for (int i = 0; i < 7; ++i) piv[i] = i;
  double c[7] = {0, 0, 0, 0, 0, 0, 0};
  double scale = 0.0;
  for (int a = 0; a < 7; ++a) scale = std::max(scale, std::fabs(M[a][a]));
  bool ok = scale > 0.0;
  for (int col = 0; col < 7 && ok; ++col) {
    int best = col;
    for (int i = col + 1; i < 7; ++i)
      if (std::fabs(M[i][col]) > std::fabs(M[best][col])) best = i;
    if (std::fabs(M[best][col]) <= 1e-13 * scale) {
      ok = false;
      break;
    }
    if (best != col) {
      for (int j = 0; j < 7; ++j) std::swap(M[col][j], M[best][j]);
      std::swap(r[col], r[best]);
    }
    for (int i = col + 1; i < 7; ++i) {
      const double f = M[i][col] / M[col][col];
      for (int j = col; j < 7; ++j) M[i][j] -= f * M[col][j];
      r[i] -= f * r[col];
    }
  }
  if (!ok) fail(CASPAR_ENUMERIC, "gauge projection: N^T D N is singular (degenerate problem)");
  for (int i = 6; i >= 0; --i) {
    double s = r[i];
    for (int j = i + 1; j < 7; ++j) s -= M[i][j] * c[j];
    c[i] = s / M[i][i];
  }
  k_gauge_apply<S><<<nblk(nb, 256), 256, 0, h->stream>>>(h->nc, h->np, h->cam, h->X, (const S*)h->vec.D,
                                                          (S*)h->vec.v, c[0], c[1], c[2], c[3], c[4], c[5], c[6]);
  CBA_LAUNCHED();
}

// Bytes the damped normal-equation product must move per launch, the figure
// its HBM roofline is priced on.  With stored blocks: per observation the
// 2x9 and 2x3 blocks (24 scalars) and two int32 indices; per parameter p and
// D read and w written.  With recomputed blocks the observation keeps only
// its two indices and the product reads the camera rows (16 scalars) and the
// float64 points instead.
double matvec_algorithmic_bytes(const caspar_ba* h) {
  const double s = (double)scalar_bytes(h->prec);
  const double per_param = 3.0 * s * (double)h->N;
  if (!h->rj) return (double)h->no * (24.0 * s + 8.0) + per_param;
  return (double)h->no * 8.0 + per_param + 24.0 * (double)h->np + 16.0 * s * (double)h->nc;
}

}  // namespace cba

using namespace cba;

#define CBA_API_BEGIN try {
#define CBA_API_END                  \
  }                                  \
  catch (const Error& e) {           \
    set_last_error(e.msg);           \
    return e.status;                 \
  }                                  \
  catch (const std::exception& e) {  \
    set_last_error(e.what());        \
    return CASPAR_EHIP;              \
  }                                  \
  set_last_error("");                \
  return CASPAR_OK;

extern "C" {

int caspar_ba_solve(caspar_ba* h, const caspar_solve_opts* opts, caspar_solve_stats* stats,
                    caspar_iter_record* history) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  check_device(h);
  solve_impl(h, opts, stats, history);
  sync(h);  // a read-back by polling leaves the stream drained already; this keeps the contract explicit
  CBA_API_END
}

int caspar_ba_linearize(caspar_ba* h, double* cost, double* resid, double* jac_cam, double* jac_pt,
                        double* grad, double* diag) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  check_device(h);
  h->linearized = false;
  run_linearize(h);
  if (resid || jac_cam || jac_pt) run_export_linearization(h, resid, jac_cam, jac_pt);
  if (grad) run_to_caller_vector(h, h->vec.g, grad);
  if (diag) run_to_caller_vector(h, h->vec.D, diag);
  if (cost) *cost = h->cost;
  sync(h);
  CBA_API_END
}

int caspar_ba_matvec(caspar_ba* h, double lambda, const double* p, double* w, double* pAp) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  CBA_REQUIRE(h->N == 0 || (p && w), "p or w is NULL");
  CBA_REQUIRE(std::isfinite(lambda) && lambda >= 0.0, "lambda must be finite and >= 0");
  check_device(h);
  ensure_linearized(h);
  run_from_caller_vector(h, p, h->vec.v);
  run_matvec(h, lambda, h->vec.v, h->vec.w, false);
  run_to_caller_vector(h, h->vec.w, w);
  const DevScalars s = read_scalars(h);
  timing_harvest(h, 1);
  if (pAp) *pAp = s.pAp;
  CBA_API_END
}

int caspar_ba_block_jacobi_apply(caspar_ba* h, double lambda, const double* r, double* z) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  CBA_REQUIRE(h->N == 0 || (r && z), "r or z is NULL");
  CBA_REQUIRE(std::isfinite(lambda) && lambda >= 0.0, "lambda must be finite and >= 0");
  check_device(h);
  ensure_linearized(h);
  run_block_jacobi(h, lambda);
  run_from_caller_vector(h, r, h->vec.v);
  run_bj_apply(h, h->vec.v, h->vec.z);
  run_to_caller_vector(h, h->vec.z, z);
  sync(h);
  CBA_API_END
}

int caspar_ba_pcg(caspar_ba* h, double lambda, const double* b, double tol, int32_t max_iters, double* x,
                  int32_t* iters, double* rel_resid) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  CBA_REQUIRE(h->N == 0 || (b && x), "b or x is NULL");
  CBA_REQUIRE(std::isfinite(lambda) && lambda >= 0.0 && tol >= 0.0 && max_iters >= 0, "bad PCG arguments");
  check_device(h);
  ensure_linearized(h);
  run_from_caller_vector(h, b, h->vec.v);
  double rel = 0.0;
  const int k = run_pcg(h, lambda, h->vec.v, false, tol, max_iters, 4, nullptr, &rel);
  run_to_caller_vector(h, h->vec.x, x);
  sync(h);
  if (iters) *iters = k;
  if (rel_resid) *rel_resid = rel;
  CBA_API_END
}

int caspar_ba_cost_fp64(caspar_ba* h, double* cost) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr && cost != nullptr, "NULL argument");
  check_device(h);
  *cost = run_cost(h, h->cam, h->X, true);
  CBA_API_END
}

int caspar_ba_set_timing(caspar_ba* h, int enable) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  CBA_REQUIRE(enable >= 0, "negative timing stride");
  h->timing_every = enable;
  h->ev_used = 0;
  h->mv_seq = 0;
  h->mv_in_solve = 0;
  if (enable > 0) {
    h->mv_launches = 0;
    h->mv_ms = 0.0;
  }
  CBA_API_END
}

int caspar_ba_get_timing(caspar_ba* h, caspar_timing* out) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr && out != nullptr, "NULL argument");
  out->matvec_launches = h->mv_launches;
  out->matvec_ms = h->mv_ms;
  out->matvec_bytes = matvec_algorithmic_bytes(h);
  CBA_API_END
}

int caspar_ba_backward(caspar_ba* h, const double* grad_cams, const double* grad_points, double lambda_adj,
                       double pcg_tol, int32_t max_pcg_iters, int32_t flags, double* grad_obs_px,
                       int32_t* pcg_iters, double* rel_resid) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  CBA_REQUIRE(h->no == 0 || grad_obs_px != nullptr, "grad_obs_px is NULL");
  CBA_REQUIRE(std::isfinite(lambda_adj) && lambda_adj > 0.0, "lambda_adj must be finite and > 0");
  CBA_REQUIRE(pcg_tol >= 0.0 && max_pcg_iters >= 0, "bad PCG arguments");
  check_device(h);
  ensure_linearized(h);
  CBA_REQUIRE((flags & ~CASPAR_ADJ_GAUGE_PROJECT) == 0, "unknown backward flags");
  CBA_REQUIRE(!(flags & CASPAR_ADJ_GAUGE_PROJECT) || h->n_between == 0,
              "gauge projection removes the similarity gauge of reprojection-only problems; "
              "pose between-factors fix the scale");
  if (h->prec == CASPAR_FP64)
    adjoint_rhs_t<double>(h, grad_cams, grad_points);
  else
    adjoint_rhs_t<float>(h, grad_cams, grad_points);
  if (flags & CASPAR_ADJ_GAUGE_PROJECT) {
    if (h->prec == CASPAR_FP64)
      gauge_project_t<double>(h);
    else
      gauge_project_t<float>(h);
  }
  double rel = 0.0;
  const int k = run_pcg(h, lambda_adj, h->vec.v, false, pcg_tol, max_pcg_iters, 4, nullptr, &rel);
  if (h->prec == CASPAR_FP64)
    adjoint_obs_t<double>(h, grad_obs_px);
  else
    adjoint_obs_t<float>(h, grad_obs_px);
  sync(h);
  if (pcg_iters) *pcg_iters = k;
  if (rel_resid) *rel_resid = rel;
  CBA_API_END
}

}  // extern "C"
