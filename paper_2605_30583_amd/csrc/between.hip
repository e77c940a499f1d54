// Pose between-factors on pairs of cameras: a second factor type beside the
// reprojection factor.  The paper generates one solver per collection of
// factor types, with an odometry factor as its example (Section V), and
// reads chain factors through pairwise accessors (Section IV-A).  Residual
// of a factor between cameras i and j with measured relative pose
// Z = (Z_R, Z_t) and square-root weights s_rot, s_trans:
//   r = [ s_rot   Log(Z_R^T R_j R_i^T) ;
//         s_trans (t_j - R_j R_i^T t_i - Z_t) ]
// (T_j T_i^-1 for world-to-camera poses).  Blocks over the camera tangent
// [dw, dt] with R <- R Exp(dw), t <- t + dt; phi = Log(Z_R^T R_j R_i^T),
// u = R_i^T t_i, Jr^-1 the inverse right Jacobian of SO(3):
//   first camera:  [[-s_rot Jr^-1(phi) R_i, 0], [-s_trans R_j [u]x, -s_trans R_j R_i^T]]
//   second camera: [[ s_rot Jr^-1(phi) R_i, 0], [ s_trans R_j [u]x,  s_trans I]]
// The calibration columns are zero.
//
// Each camera gathers its incident factors through a host-built incidence
// list (the pairwise read: both cameras of a factor) and adds its own side's
// share (the pairwise add, with no atomics).  The linearisation evaluates
// every factor in float64 at both endpoints and keeps its blocks; each
// product applies the kept blocks.  Factors are few (about one per camera),
// so the kernels are small beside the reprojection work.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"
#include "model.hpp"

namespace cba {

// Blocks of a factor kept from the linearisation for the products: with
// Ji = [[-A, 0], [-B, -C]] and Jj = [[A, 0], [B, s_trans I]] only A, B, C
// (row-major) and s_trans are stored.
constexpr int kBetweenBlock = 28;

// Residual (and with BLOCKS the two 6x6 blocks, columns [dw, dt]) of factor
// F at the float64 camera rows.
template <bool BLOCKS>
__device__ inline void between_eval(const BetweenFactor& F, const double* __restrict__ cam, double r[6],
                                    double Ji[6][6], double Jj[6][6]) {
  const double* a = cam + (size_t)F.ci * kCamStride;
  const double* b = cam + (size_t)F.cj * kCamStride;
  double Ri[9], Rj[9], ti[3], tj[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    Ri[k] = a[k];
    Rj[k] = b[k];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ti[k] = a[9 + k];
    tj[k] = b[9 + k];
  }
  // Rij = R_j R_i^T, E = Z_R^T Rij
  double Rij[9], E[9];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y)
      Rij[3 * x + y] = Rj[3 * x] * Ri[3 * y] + Rj[3 * x + 1] * Ri[3 * y + 1] + Rj[3 * x + 2] * Ri[3 * y + 2];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y)
      E[3 * x + y] = F.ZR[x] * Rij[y] + F.ZR[3 + x] * Rij[3 + y] + F.ZR[6 + x] * Rij[6 + y];
  double phi[3];
  so3_log(E, phi);
  // u = R_i^T t_i; R_j R_i^T t_i = R_j u
  double u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = Ri[k] * ti[0] + Ri[3 + k] * ti[1] + Ri[6 + k] * ti[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = F.s_rot * phi[k];
    const double Rju = Rj[3 * k] * u[0] + Rj[3 * k + 1] * u[1] + Rj[3 * k + 2] * u[2];
    r[3 + k] = F.s_trans * (tj[k] - Rju - F.Zt[k]);
  }
  if (!BLOCKS) return;
  // Jr^-1(phi) = I + 1/2 [phi]x + c [phi]x^2, c = 1/a^2 - cot(a/2) / (2a)
  const double a2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  double c;
  if (a2 < 1e-6) {
    c = 1.0 / 12.0 + a2 / 720.0;
  } else {
    const double an = sqrt(a2);
    c = 1.0 / a2 - 1.0 / (2.0 * an * tan(0.5 * an));
  }
  const double K[9] = {0.0, -phi[2], phi[1], phi[2], 0.0, -phi[0], -phi[1], phi[0], 0.0};
  double M[9];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      // [phi]x^2 = phi phi^T - a2 I
      const double K2 = phi[x] * phi[y] - (x == y ? a2 : 0.0);
      M[3 * x + y] = (x == y ? 1.0 : 0.0) + 0.5 * K[3 * x + y] + c * K2;
    }
  const double Ux[9] = {0.0, -u[2], u[1], u[2], 0.0, -u[0], -u[1], u[0], 0.0};
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const double A = F.s_rot * (M[3 * x] * Ri[y] + M[3 * x + 1] * Ri[3 + y] + M[3 * x + 2] * Ri[6 + y]);
      const double B = F.s_trans * (Rj[3 * x] * Ux[y] + Rj[3 * x + 1] * Ux[3 + y] + Rj[3 * x + 2] * Ux[6 + y]);
      const double C = F.s_trans * Rij[3 * x + y];
      Ji[x][y] = -A;
      Jj[x][y] = A;
      Ji[x][3 + y] = 0.0;
      Jj[x][3 + y] = 0.0;
      Ji[3 + x][y] = -B;
      Jj[3 + x][y] = B;
      Ji[3 + x][3 + y] = -C;
      Jj[3 + x][3 + y] = x == y ? F.s_trans : 0.0;
    }
}

// Linearisation: per camera, g_c += J_c^T r and H_cc += J_c^T J_c over its
// incident factors (the [dw, dt] part), then D_c for those six columns from
// the updated diagonal.  Partials: sum of r.r, each factor counted at its
// first camera.  Runs after the reprojection sums are in g, H_cc and D.
template <typename S>
__global__ __launch_bounds__(64) void k_between_lin(int nc, const double* __restrict__ cam,
                                                     const BetweenFactor* __restrict__ fac,
                                                     const int* __restrict__ off, const int* __restrict__ inc,
                                                     S* __restrict__ g, S* __restrict__ D, double* __restrict__ Hcc,
                                                     double* __restrict__ blocks, double* __restrict__ partials) {
  __shared__ double red[4];
  double rr = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    const int q0 = off[c], q1 = off[c + 1];
    if (q0 == q1) continue;
    double g6[6] = {0, 0, 0, 0, 0, 0}, H[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) H[k] = 0.0;
    for (int q = q0; q < q1; ++q) {
      const int e = inc[q];
      const BetweenFactor F = fac[e >> 1];
      double r[6], Ji[6][6], Jj[6][6];
      between_eval<true>(F, cam, r, Ji, Jj);
      const bool second = (e & 1) != 0;
      if (!second) {
        rr += r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3] + r[4] * r[4] + r[5] * r[5];
        // the factor's blocks for the products, written once (first camera)
        double* bl = blocks + (size_t)(e >> 1) * kBetweenBlock;
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
          for (int y = 0; y < 3; ++y) {
            bl[3 * x + y] = Jj[x][y];
            bl[9 + 3 * x + y] = Jj[3 + x][y];
            bl[18 + 3 * x + y] = -Ji[3 + x][3 + y];
          }
        bl[27] = F.s_trans;
      }
      int t = 0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int a = 0; a < 6; ++a) g6[k] += (second ? Jj[a][k] : Ji[a][k]) * r[a];
#pragma unroll
        for (int l = k; l < 6; ++l, ++t) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < 6; ++a) s += (second ? Jj[a][k] * Jj[a][l] : Ji[a][k] * Ji[a][l]);
          H[t] += s;
        }
      }
    }
    int t = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const size_t gi = 9 * (size_t)c + k;
      g[gi] = (S)((double)g[gi] + g6[k]);
#pragma unroll
      for (int l = k; l < 6; ++l, ++t) Hcc[45 * (size_t)c + tri9(k, l)] += H[t];
      D[gi] = (S)clamp_diag(Hcc[45 * (size_t)c + tri9(k, k)]);
    }
  }
  const double s = block_sum(rr, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kPartialWidth] = s;
}

// Sum of r.r over the factors at camera rows `cam` (trial cost, float64 cost).
__global__ __launch_bounds__(256) void k_between_cost(int nf, const double* __restrict__ cam,
                                                      const BetweenFactor* __restrict__ fac,
                                                      double* __restrict__ partials) {
  __shared__ double red[4];
  double rr = 0.0;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += gridDim.x * blockDim.x) {
    double r[6];
    between_eval<false>(fac[f], cam, r, nullptr, nullptr);
#pragma unroll
    for (int k = 0; k < 6; ++k) rr += r[k] * r[k];
  }
  const double s = block_sum(rr, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kPartialWidth] = s;
}

// Product: per camera, rows[c] = sum over its factors of J_c^T (J_i p_i + J_j p_j)
// (the [dw, dt] part; the final product kernel adds it to w), and the
// partials of |J_i p_i + J_j p_j|^2, each factor counted at its first camera.
// With the stored A, B, C: q_rot = A (w_j - w_i), q_trans = B (w_j - w_i) -
// C t_i + s_trans t_j for the [dw, dt] parts w, t of p; the first camera
// takes (-A^T q_rot - B^T q_trans, -C^T q_trans), the second
// (A^T q_rot + B^T q_trans, s_trans q_trans).
template <typename S>
__global__ __launch_bounds__(64) void k_between_product(int nc, const BetweenFactor* __restrict__ fac,
                                                         const double* __restrict__ blocks,
                                                         const int* __restrict__ off, const int* __restrict__ inc,
                                                         const S* __restrict__ p, double* __restrict__ rows,
                                                         double* __restrict__ partials,
                                                         const DevScalars* __restrict__ sc) {
  __shared__ double red[4];
  if (sc != nullptr && sc->done) return;
  double pap = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    double w6[6] = {0, 0, 0, 0, 0, 0};
    for (int q = off[c]; q < off[c + 1]; ++q) {
      const int e = inc[q];
      const int f = e >> 1;
      const int ci = fac[f].ci, cj = fac[f].cj;
      const double* bl = blocks + (size_t)f * kBetweenBlock;
      double dw[3], ti[3], tj[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        dw[k] = (double)p[9 * (size_t)cj + k] - (double)p[9 * (size_t)ci + k];
        ti[k] = (double)p[9 * (size_t)ci + 3 + k];
        tj[k] = (double)p[9 * (size_t)cj + 3 + k];
      }
      const double st = bl[27];
      double qr[3], qt[3];
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        qr[x] = bl[3 * x] * dw[0] + bl[3 * x + 1] * dw[1] + bl[3 * x + 2] * dw[2];
        qt[x] = bl[9 + 3 * x] * dw[0] + bl[9 + 3 * x + 1] * dw[1] + bl[9 + 3 * x + 2] * dw[2] -
                (bl[18 + 3 * x] * ti[0] + bl[18 + 3 * x + 1] * ti[1] + bl[18 + 3 * x + 2] * ti[2]) + st * tj[x];
      }
      const bool second = (e & 1) != 0;
      if (!second) pap += qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qt[0] * qt[0] + qt[1] * qt[1] + qt[2] * qt[2];
      const double sg = second ? 1.0 : -1.0;
#pragma unroll
      for (int y = 0; y < 3; ++y) {
        const double aq = bl[y] * qr[0] + bl[3 + y] * qr[1] + bl[6 + y] * qr[2];
        const double bq = bl[9 + y] * qt[0] + bl[12 + y] * qt[1] + bl[15 + y] * qt[2];
        const double cq = bl[18 + y] * qt[0] + bl[21 + y] * qt[1] + bl[24 + y] * qt[2];
        w6[y] += sg * (aq + bq);
        w6[3 + y] += second ? st * qt[y] : -cq;
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) rows[6 * (size_t)c + k] = w6[k];
  }
  const double s = block_sum(pap, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kPartialWidth] = s;
}

__global__ void k_between_sum(int n, const double* __restrict__ partials, DevScalars* sc, int slot) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[(size_t)i * kPartialWidth];
  s = block_sum(s, red);
  if (threadIdx.x == 0) sc->red[slot] = s;
}

// One wave per workgroup: a camera's factors run one after another in its
// thread, so the cameras are spread over as many CUs as there are waves.
constexpr int kBetweenThreads = 64;

unsigned between_grid(const caspar_ba* h) {
  return (unsigned)std::max(1, std::min((h->nc + kBetweenThreads - 1) / kBetweenThreads, 1024));
}

void run_between_lin(caspar_ba* h) {
  if (h->n_between == 0) return;
  const unsigned g = between_grid(h);
  if (h->prec == CASPAR_FP64)
    k_between_lin<double><<<g, kBetweenThreads, 0, h->stream>>>(h->nc, h->cam, h->between, h->bt_off, h->bt_inc,
                                                   (double*)h->vec.g, (double*)h->vec.D, h->Hcc, h->bt_blocks,
                                                   h->partials);
  else
    k_between_lin<float><<<g, kBetweenThreads, 0, h->stream>>>(h->nc, h->cam, h->between, h->bt_off, h->bt_inc,
                                                  (float*)h->vec.g, (float*)h->vec.D, h->Hcc, h->bt_blocks,
                                                  h->partials);
  CBA_LAUNCHED();
  k_between_sum<<<1, 1024, 0, h->stream>>>((int)g, h->partials, h->scal, 7);
  CBA_LAUNCHED();
}

void launch_between_cost(caspar_ba* h, const double* cam) {
  if (h->n_between == 0) return;
  const unsigned g = (unsigned)std::max(1, std::min((h->n_between + 255) / 256, 1024));
  k_between_cost<<<g, 256, 0, h->stream>>>(h->n_between, cam, h->between, h->partials);
  CBA_LAUNCHED();
  k_between_sum<<<1, 1024, 0, h->stream>>>((int)g, h->partials, h->scal, 7);
  CBA_LAUNCHED();
}

double run_between_cost(caspar_ba* h, const double* cam) {
  if (h->n_between == 0) return 0.0;
  launch_between_cost(h, cam);
  return 0.5 * read_scalars(h).red[7];
}

void run_between_product(caspar_ba* h, const void* p, bool pcg_mode) {
  if (h->n_between == 0) return;
  const DevScalars* scp = pcg_mode ? h->scal : nullptr;
  // partial slots after the fused product's G workgroup slots
  double* part = h->partials + (size_t)h->G * kPartialWidth;
  if (h->prec == CASPAR_FP64)
    k_between_product<double><<<between_grid(h), kBetweenThreads, 0, h->stream>>>(
        h->nc, h->between, h->bt_blocks, h->bt_off, h->bt_inc, (const double*)p, h->bt_rows, part, scp);
  else
    k_between_product<float><<<between_grid(h), kBetweenThreads, 0, h->stream>>>(
        h->nc, h->between, h->bt_blocks, h->bt_off, h->bt_inc, (const float*)p, h->bt_rows, part, scp);
  CBA_LAUNCHED();
}

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct BetweenPlan {
  size_t fac, off, inc, rows, blocks, total;
};

BetweenPlan between_plan(int64_t n, int64_t nc) {
  BetweenPlan p{};
  size_t o = 0;
  p.fac = o;
  o += align256((size_t)n * sizeof(BetweenFactor));
  p.off = o;
  o += align256((size_t)(nc + 1) * sizeof(int));
  p.inc = o;
  o += align256((size_t)(2 * n) * sizeof(int));
  p.rows = o;
  o += align256((size_t)nc * 6 * sizeof(double));
  p.blocks = o;
  o += align256((size_t)n * kBetweenBlock * sizeof(double));
  p.total = o;
  return p;
}

// Rotation matrix of an angle-axis vector (Rodrigues, float64), row-major.
void host_so3_exp(const double w[3], double R[9]) {
  const double a2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double s, c;
  if (a2 < 1e-8) {
    s = 1.0 - a2 / 6.0 + a2 * a2 / 120.0;
    c = 0.5 - a2 / 24.0 + a2 * a2 / 720.0;
  } else {
    const double a = std::sqrt(a2);
    s = std::sin(a) / a;
    c = (1.0 - std::cos(a)) / a2;
  }
  const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y) {
      const double K2 = w[x] * w[y] - (x == y ? a2 : 0.0);
      R[3 * x + y] = (x == y ? 1.0 : 0.0) + s * K[3 * x + y] + c * K2;
    }
}

}  // namespace
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

size_t caspar_ba_between_workspace_bytes(int32_t n_factors, int32_t n_cams) {
  if (n_factors < 0 || n_cams < 0) return 0;
  return between_plan(n_factors, n_cams).total;
}

int caspar_ba_set_between(caspar_ba* h, int32_t n_factors, const int32_t* cam_i, const int32_t* cam_j,
                          const double* meas, const double* weights, void* dev_workspace, size_t workspace_bytes) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "null handle");
  CBA_REQUIRE(n_factors >= 0, "negative number of between-factors");
  if (n_factors == 0) {
    h->n_between = 0;
    h->between = nullptr;
    h->bt_off = h->bt_inc = nullptr;
    h->bt_rows = nullptr;
    h->bt_blocks = nullptr;
    h->linearized = false;
    h->bj_lambda = -1.0;
    return CASPAR_OK;
  }
  CBA_REQUIRE(cam_i && cam_j && meas && weights, "null between-factor array");
  const BetweenPlan plan = between_plan(n_factors, h->nc);
  CBA_REQUIRE(dev_workspace != nullptr && workspace_bytes >= plan.total,
              "between workspace smaller than caspar_ba_between_workspace_bytes()");
  CBA_REQUIRE((reinterpret_cast<uintptr_t>(dev_workspace) & 255) == 0, "between workspace must be 256-byte aligned");
  for (int32_t f = 0; f < n_factors; ++f) {
    CBA_REQUIRE(cam_i[f] >= 0 && cam_i[f] < h->nc && cam_j[f] >= 0 && cam_j[f] < h->nc,
                "between-factor " + std::to_string(f) + ": camera index out of range");
    CBA_REQUIRE(cam_i[f] != cam_j[f], "between-factor " + std::to_string(f) + ": both cameras are the same");
    for (int k = 0; k < 6; ++k)
      CBA_REQUIRE(std::isfinite(meas[6 * (size_t)f + k]),
                  "between-factor " + std::to_string(f) + ": non-finite measurement");
    for (int k = 0; k < 2; ++k)
      CBA_REQUIRE(std::isfinite(weights[2 * (size_t)f + k]) && weights[2 * (size_t)f + k] > 0.0,
                  "between-factor " + std::to_string(f) + ": weights must be finite and positive");
  }
  // caller -> internal camera ids
  std::vector<int> c2i(h->nc);
  CBA_HIP(hipMemcpyAsync(c2i.data(), h->cam_c2i, sizeof(int) * (size_t)h->nc, hipMemcpyDeviceToHost, h->stream));
  CBA_HIP(hipStreamSynchronize(h->stream));
  std::vector<BetweenFactor> fac(n_factors);
  std::vector<int> cnt(h->nc + 1, 0);
  for (int32_t f = 0; f < n_factors; ++f) {
    BetweenFactor& F = fac[f];
    F.ci = c2i[cam_i[f]];
    F.cj = c2i[cam_j[f]];
    host_so3_exp(meas + 6 * (size_t)f, F.ZR);
    for (int k = 0; k < 3; ++k) F.Zt[k] = meas[6 * (size_t)f + 3 + k];
    F.s_rot = weights[2 * (size_t)f];
    F.s_trans = weights[2 * (size_t)f + 1];
    F.pad = 0.0;
    ++cnt[F.ci + 1];
    ++cnt[F.cj + 1];
  }
  for (int c = 0; c < h->nc; ++c) cnt[c + 1] += cnt[c];
  std::vector<int> inc(2 * (size_t)n_factors), pos(cnt.begin(), cnt.end() - 1);
  for (int32_t f = 0; f < n_factors; ++f) {
    inc[pos[fac[f].ci]++] = 2 * f;
    inc[pos[fac[f].cj]++] = 2 * f + 1;
  }
  char* ws = static_cast<char*>(dev_workspace);
  CBA_HIP(hipMemcpyAsync(ws + plan.fac, fac.data(), sizeof(BetweenFactor) * fac.size(), hipMemcpyHostToDevice,
                         h->stream));
  CBA_HIP(hipMemcpyAsync(ws + plan.off, cnt.data(), sizeof(int) * cnt.size(), hipMemcpyHostToDevice, h->stream));
  CBA_HIP(hipMemcpyAsync(ws + plan.inc, inc.data(), sizeof(int) * inc.size(), hipMemcpyHostToDevice, h->stream));
  CBA_HIP(hipStreamSynchronize(h->stream));
  h->n_between = n_factors;
  h->between = reinterpret_cast<BetweenFactor*>(ws + plan.fac);
  h->bt_off = reinterpret_cast<int*>(ws + plan.off);
  h->bt_inc = reinterpret_cast<int*>(ws + plan.inc);
  h->bt_rows = reinterpret_cast<double*>(ws + plan.rows);
  h->bt_blocks = reinterpret_cast<double*>(ws + plan.blocks);
  h->linearized = false;
  h->bj_lambda = -1.0;
  CBA_API_END
}

}  // extern "C"
