// Fused damped normal-equation product w = (J^T J + lambda D) p and
// p^T w = |J p|^2 + lambda p^T D p, matrix-free (Section V: the normal
// equations are solved directly; J^T J is never formed).
//
// Per observation o with camera c and point j:  q_o = J_c,o p_c + J_j,o p_j,
// camera contribution J_c,o^T q_o (9), point contribution J_j,o^T q_o (3).
//
// The paper's shared-add accessor (Section IV-A) reduces per block and then
// issues one global atomic per unique index.  On MI355X global FP64 atomics
// sustain only ~22 G/s, far below the rate observations stream in, so this
// kernel keeps all camera accumulation on chip instead:
//  * persistent workgroups (1024 threads) each own a contiguous range of wave
//    tiles and keep float64 accumulators for the K most observed cameras in
//    LDS (ds_add_f64), flushed once per workgroup as plain rows;
//  * observations of the remaining cameras write their 9-vector to a row of
//    their own (ballot-ranked inside the wave, so rows stay coalesced);
//  * points are contiguous inside a tile: an in-wave segmented scan sums their
//    contributions and the first lane of each point writes w_j directly.
// A second small kernel adds the per-workgroup rows and cold rows of each
// camera (fixed order: deterministic), handles split and orphan points and
// turns the p^T A p partials into alpha for PCG.
#include "common.hpp"
#include "model.hpp"

namespace cba {

template <typename S>
__global__ __launch_bounds__(kMvThreads) void k_matvec(
    int n_tiles, int G, const Tile* __restrict__ tiles, const uint32_t* __restrict__ meta,
    const void* __restrict__ J, int no_pad, const S* __restrict__ p, const S* __restrict__ D,
    double lambda, S* __restrict__ w, int nc, int K, int n_orphan, double* __restrict__ hot_rows,
    double* __restrict__ cold_rows, double* __restrict__ split_rows, double* __restrict__ partials,
    const DevScalars* __restrict__ sc) {
  extern __shared__ double hot[];  // [K][9]
  __shared__ double red[kMvWaves];
  if (sc != nullptr && sc->done) return;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  for (int i = tid; i < K * 9; i += kMvThreads) hot[i] = 0.0;
  __syncthreads();

  const S* __restrict__ pp_base = p + 9 * (size_t)nc;
  const S* __restrict__ dp_base = D + 9 * (size_t)nc;
  S* __restrict__ wp_base = w + 9 * (size_t)nc;
  double pap = 0.0;
  const int t0 = (int)((int64_t)n_tiles * blockIdx.x / G);
  const int t1 = (int)((int64_t)n_tiles * (blockIdx.x + 1) / G);
  for (int t = t0 + wv; t < t1; t += kMvWaves) {
    const Tile tl = tiles[t];
    const int n = tile_nobs(tl.info);
    const bool act = lane < n;
    int lp = 100 + lane;
    int ci = -1;
    S yc[9], yp[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) yc[k] = (S)0;
#pragma unroll
    for (int k = 0; k < 3; ++k) yp[k] = (S)0;
    if (act) {
      const int o = tl.obs_begin + lane;
      const uint32_t m = meta[o];
      ci = (int)(m & ((1u << kCamBits) - 1));
      lp = (int)(m >> kCamBits);
      S col[12][2];
      JStore<S>::load(J, no_pad, o, col);
      const S* pc = p + 9 * (size_t)ci;
      const S* pj = pp_base + 3 * (size_t)(tl.pt_begin + lp);
      S q0 = (S)0, q1 = (S)0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const S v = pc[k];
        q0 = fma(col[k][0], v, q0);
        q1 = fma(col[k][1], v, q1);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const S v = pj[k];
        q0 = fma(col[9 + k][0], v, q0);
        q1 = fma(col[9 + k][1], v, q1);
      }
      pap = fma((double)q0, (double)q0, fma((double)q1, (double)q1, pap));
#pragma unroll
      for (int k = 0; k < 9; ++k) yc[k] = fma(col[k][0], q0, col[k][1] * q1);
#pragma unroll
      for (int k = 0; k < 3; ++k) yp[k] = fma(col[9 + k][0], q0, col[9 + k][1] * q1);
      if (ci < K) {
        double* a = hot + 9 * ci;
#pragma unroll
        for (int k = 0; k < 9; ++k) atomicAdd(a + k, (double)yc[k]);
      }
    }
    // cameras outside the LDS set: one row per observation
    const bool cold = act && ci >= K;
    const unsigned long long cm = __ballot(cold);
    if (cold) {
      const int rank = __popcll(cm & ((1ull << lane) - 1ull));
      double* row = cold_rows + (size_t)(tl.cold_begin + rank) * 9;
#pragma unroll
      for (int k = 0; k < 9; ++k) row[k] = (double)yc[k];
    }
    // points: segmented suffix sums, the first lane of each point holds the total
    const int steps = tile_steps(tl.info);
    for (int s = 0, d = 1; s < steps; ++s, d <<= 1) {
      const int olp = __shfl_down(lp, d, kWave);
      const bool take = (lane + d < kWave) && olp == lp;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const S o = __shfl_down(yp[k], d, kWave);
        if (take) yp[k] += o;
      }
    }
    const int prev = __shfl_up(lp, 1, kWave);
    const bool head = act && (lane == 0 || prev != lp);
    if (head) {
      const size_t b = 3 * (size_t)(tl.pt_begin + lp);
      if (tile_split(tl.info)) {
        double* row = split_rows + (size_t)tl.split_row * kPtRowWidth;
#pragma unroll
        for (int k = 0; k < 3; ++k) row[k] = (double)yp[k];
        if (tile_first(tl.info)) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double v = pp_base[b + k];
            pap = fma(lambda * (double)dp_base[b + k] * v, v, pap);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const S v = pp_base[b + k];
          const S dv = dp_base[b + k];
          wp_base[b + k] = fma((S)lambda * dv, v, yp[k]);
          pap = fma(lambda * (double)dv * (double)v, (double)v, pap);
        }
      }
    }
  }
  // lambda p^T D p of the camera blocks and of points without observations
  for (int i = blockIdx.x * kMvThreads + tid; i < 9 * nc; i += G * kMvThreads) {
    const double v = p[i];
    pap = fma(lambda * (double)D[i] * v, v, pap);
  }
  for (int i = blockIdx.x * kMvThreads + tid; i < 3 * n_orphan; i += G * kMvThreads) {
    const double v = pp_base[i];
    pap = fma(lambda * (double)dp_base[i] * v, v, pap);
  }
  const double tot = block_sum(pap, red);
  if (tid == 0) partials[(size_t)blockIdx.x * kPartialWidth] = tot;
  double* dst = hot_rows + (size_t)blockIdx.x * K * 9;
  for (int i = tid; i < K * 9; i += kMvThreads) dst[i] = hot[i];
}

// Camera rows of w, split and orphan points, p^T A p and (in PCG) alpha.
template <typename S>
__global__ __launch_bounds__(256) void k_matvec_final(
    int nc, int K, int G, const double* __restrict__ hot_rows, const double* __restrict__ cold_rows,
    const int* __restrict__ cold_off, const int* __restrict__ cold_list, const S* __restrict__ p,
    const S* __restrict__ D, double lambda, S* __restrict__ w, int n_split,
    const SplitPoint* __restrict__ sp, const double* __restrict__ split_rows, int n_orphan,
    const double* __restrict__ partials, DevScalars* __restrict__ sc, int pcg_mode) {
  __shared__ double red[4];
  if (pcg_mode && sc->done) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ncam = 9 * (int64_t)nc;
  const int64_t nsplit = 3 * (int64_t)n_split;
  if (i < ncam) {
    const int c = (int)(i / 9), k = (int)(i % 9);
    double s = 0.0;
    if (c < K) {
      const double* r = hot_rows + (size_t)c * 9 + k;
      const size_t stride = (size_t)K * 9;
      for (int g = 0; g < G; ++g) s += r[g * stride];
    } else {
      const int b = cold_off[c - K], e = cold_off[c - K + 1];
      for (int q = b; q < e; ++q) s += cold_rows[(size_t)cold_list[q] * 9 + k];
    }
    w[i] = (S)fma(lambda * (double)D[i], (double)p[i], s);
  } else if (i < ncam + nsplit) {
    const int64_t jx = i - ncam;
    const SplitPoint s = sp[jx / 3];
    const int k = (int)(jx % 3);
    double acc = 0.0;
    for (int r = 0; r < s.nrows; ++r) acc += split_rows[(size_t)(s.row_begin + r) * kPtRowWidth + k];
    const size_t b = 9 * (size_t)nc + 3 * (size_t)s.pt + k;
    w[b] = (S)fma(lambda * (double)D[b], (double)p[b], acc);
  } else if (i < ncam + nsplit + 3 * (int64_t)n_orphan) {
    const size_t b = 9 * (size_t)nc + (size_t)(i - ncam - nsplit);
    w[b] = (S)(lambda * (double)D[b] * (double)p[b]);
  }
  if (blockIdx.x == 0) {
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += blockDim.x) s += partials[(size_t)g * kPartialWidth];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
      sc->pAp = s;
      if (pcg_mode) {
        sc->iter += 1;
        if (!(s > 0.0) || !isfinite(s)) {
          sc->done = 1;
          sc->reason = PCG_BREAKDOWN;
        } else {
          sc->alpha = sc->rho / s;
        }
      }
    }
  }
}

template <typename S>
static void matvec_t(caspar_ba* h, double lambda, const S* p, S* w, bool pcg_mode) {
  hipStream_t st = h->stream;
  const size_t lds = (size_t)h->K * 9 * sizeof(double);
  const DevScalars* scp = pcg_mode ? h->scal : nullptr;
  if (h->n_tiles > 0 || h->nc > 0 || h->n_orphan_pts > 0) {
    k_matvec<S><<<h->G, kMvThreads, lds, st>>>(h->n_tiles, h->G, h->tiles, h->meta, h->J, h->no_pad, p,
                                                (const S*)h->vec.D, lambda, w, h->nc, h->K, h->n_orphan_pts,
                                                h->hot_rows, h->cold_rows, h->split_rows, h->partials, scp);
    CBA_LAUNCHED();
  }
  const int64_t n = 9 * (int64_t)h->nc + 3 * (int64_t)h->n_split_pts + 3 * (int64_t)h->n_orphan_pts;
  const unsigned grid = (unsigned)std::max<int64_t>(1, (n + 255) / 256);
  k_matvec_final<S><<<grid, 256, 0, st>>>(h->nc, h->K, h->G, h->hot_rows, h->cold_rows, h->cold_off,
                                          h->cold_list, p, (const S*)h->vec.D, lambda, w, h->n_split_pts,
                                          h->split_pts, h->split_rows, h->n_orphan_pts, h->partials, h->scal,
                                          pcg_mode ? 1 : 0);
  CBA_LAUNCHED();
}

void run_matvec(caspar_ba* h, double lambda, const void* p, void* w, bool pcg_mode) {
  const int lds = h->K * 9 * (int)sizeof(double);
  if (h->prec == CASPAR_FP64) {
    if (lds > 65536)
      CBA_HIP(hipFuncSetAttribute((const void*)k_matvec<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kLdsBudget));
    matvec_t<double>(h, lambda, (const double*)p, (double*)w, pcg_mode);
  } else {
    if (lds > 65536)
      CBA_HIP(hipFuncSetAttribute((const void*)k_matvec<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kLdsBudget));
    matvec_t<float>(h, lambda, (const float*)p, (float*)w, pcg_mode);
  }
}

}  // namespace cba
