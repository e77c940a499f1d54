// Linearisation of the Snavely problem (paper Section VI-A factor, Section V
// tangent-space linearisation), the trial cost of the LM step and the
// retraction theta (+) delta.
//
// Point-major pass (one wave per tile of <= 64 observations): residuals,
// Jacobian blocks written once in a blocked structure-of-arrays (16-byte
// chunks of two Jacobian columns x two rows for float64, four columns for
// float32), the cost, and the point blocks g_p = J_p^T r, H_pp = J_p^T J_p
// reduced with an in-wave segmented scan (points are contiguous inside a
// tile).
// Camera-major pass (one workgroup per chunk of <= 2048 observations of one
// camera): recomputes r and J_c from the parameters and sums g_c = J_c^T r
// and the upper triangle of H_cc = J_c^T J_c without atomics.
#include "common.hpp"
#include "model.hpp"

namespace cba {

// Camera table in the working precision (used when the Jacobian is
// recomputed; the conversion matches the one the linearisation applies).
template <typename S>
__global__ void k_cam_cast(int n, const double* __restrict__ cam, S* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (S)cam[i];
}

// Camera parameters of the recomputed-block product's rows (the first
// kProdCamP values; the product's input fills the rest).  The unit quaternion
// of R is taken with the largest of the four pivots 1 + tr R, 1 + 2 R_ii - tr R
// (Shepperd's method), which keeps the division away from zero, and is
// normalised in float64 before the cast.
template <typename S>
__global__ void k_cam_quat(int nc, const double* __restrict__ cam, S* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double* in = cam + (size_t)c * kCamStride;
  const double r00 = in[0], r01 = in[1], r02 = in[2];
  const double r10 = in[3], r11 = in[4], r12 = in[5];
  const double r20 = in[6], r21 = in[7], r22 = in[8];
  const double tr = r00 + r11 + r22;
  double q[4];  // w, x, y, z
  if (tr >= r00 && tr >= r11 && tr >= r22) {
    const double s = 2.0 * sqrt(1.0 + tr);  // 4 w
    q[0] = 0.25 * s;
    q[1] = (r21 - r12) / s;
    q[2] = (r02 - r20) / s;
    q[3] = (r10 - r01) / s;
  } else if (r00 >= r11 && r00 >= r22) {
    const double s = 2.0 * sqrt(1.0 + r00 - r11 - r22);  // 4 x
    q[0] = (r21 - r12) / s;
    q[1] = 0.25 * s;
    q[2] = (r01 + r10) / s;
    q[3] = (r02 + r20) / s;
  } else if (r11 >= r22) {
    const double s = 2.0 * sqrt(1.0 - r00 + r11 - r22);  // 4 y
    q[0] = (r02 - r20) / s;
    q[1] = (r01 + r10) / s;
    q[2] = 0.25 * s;
    q[3] = (r12 + r21) / s;
  } else {
    const double s = 2.0 * sqrt(1.0 - r00 - r11 + r22);  // 4 z
    q[0] = (r10 - r01) / s;
    q[1] = (r02 + r20) / s;
    q[2] = (r12 + r21) / s;
    q[3] = 0.25 * s;
  }
  const double inv = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  S* o = out + (size_t)c * kProdCamRow;
#pragma unroll
  for (int k = 0; k < 4; ++k) o[k] = (S)(q[k] * inv);
#pragma unroll
  for (int k = 0; k < 6; ++k) o[4 + k] = (S)in[9 + k];
}

// float32 point rows (x, y, z, 0), one 16-byte load each.
__global__ void k_point_cast(int np, const double* __restrict__ X, float4* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) out[i] = make_float4((float)X[3 * (size_t)i], (float)X[3 * (size_t)i + 1], (float)X[3 * (size_t)i + 2], 0.f);
}

// ---------------------------------------------------------------------------
// Point-major linearisation.
// ---------------------------------------------------------------------------
template <typename S, bool STORE_J>
__global__ __launch_bounds__(256) void k_lin_points(int n_tiles, const Tile* __restrict__ tiles,
                                                    const uint32_t* __restrict__ meta,
                                                    const S* __restrict__ px,
                                                    const S* __restrict__ camtab,
                                                    const S* __restrict__ pts, void* J,
                                                    S* __restrict__ g, S* __restrict__ D,
                                                    double* __restrict__ Hpp,
                                                    double* __restrict__ split_rows, int nc,
                                                    double* __restrict__ partials, int loss, double loss_c,
                                                    S* __restrict__ wts) {
  __shared__ double red[4];
  const int lane = threadIdx.x & (kWave - 1);
  // wave-uniform tile index: descriptors come through the scalar cache
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int stride = gridDim.x * 4;
  double cost = 0.0;
  // One tile from its loaded inputs: residual, blocks (stored if STORE_J),
  // cost, and per point the segmented sums of g_p and the upper triangle of
  // H_p, written by the point's first lane.
  using P2 = typename Pair<S>::type;
  auto tile = [&](const Tile& tl, int n, uint32_t m, const Cam<S>& c, const S (&Xp)[3], P2 q, int o) {
    const bool act = lane < n;
    const int lp = act ? (int)(m >> kCamBits) : 100 + lane;
    double v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = 0.0;
    if (act) {
      S r0, r1, col[12][2];
      snavely_jacobian<S>(c, Xp[0], Xp[1], Xp[2], (S)q.x, (S)q.y, r0, r1, col);
      if (loss == CASPAR_LOSS_TRIVIAL) {
        cost = fma((double)r0, (double)r0, fma((double)r1, (double)r1, cost));
      } else {
        // robust loss: cost rho(s); residual and blocks scaled by sqrt(rho'(s))
        double w;
        cost += robust_rho(loss, loss_c, fma((double)r0, (double)r0, (double)r1 * (double)r1), w);
        const S sw = (S)sqrt(w);
        r0 *= sw;
        r1 *= sw;
#pragma unroll
        for (int j = 0; j < 12; ++j) {
          col[j][0] *= sw;
          col[j][1] *= sw;
        }
        wts[o] = (S)w;
      }
      if (STORE_J) JStore<S>::store(J, o, col);
      double jp[3][2];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        jp[k][0] = col[9 + k][0];
        jp[k][1] = col[9 + k][1];
        v[k] = fma(jp[k][0], (double)r0, jp[k][1] * (double)r1);
      }
      v[3] = fma(jp[0][0], jp[0][0], jp[0][1] * jp[0][1]);
      v[4] = fma(jp[0][0], jp[1][0], jp[0][1] * jp[1][1]);
      v[5] = fma(jp[0][0], jp[2][0], jp[0][1] * jp[2][1]);
      v[6] = fma(jp[1][0], jp[1][0], jp[1][1] * jp[1][1]);
      v[7] = fma(jp[1][0], jp[2][0], jp[1][1] * jp[2][1]);
      v[8] = fma(jp[2][0], jp[2][0], jp[2][1] * jp[2][1]);
    }
    // segmented suffix sums: the first lane of each point ends with its total
    const int steps = tile_steps(tl.info);
    for (int s = 0, d = 1; s < steps; ++s, d <<= 1) {
      const int olp = __shfl_down(lp, d, kWave);
      const bool take = (lane + d < kWave) && olp == lp;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const double ov = __shfl_down(v[k], d, kWave);
        if (take) v[k] += ov;
      }
    }
    const int prev = __shfl_up(lp, 1, kWave);
    const bool head = act && (lane == 0 || prev != lp);
    if (head) {
      if (tile_split(tl.info)) {
        double* row = split_rows + (size_t)tl.split_row * kPtRowWidth;
#pragma unroll
        for (int k = 0; k < 9; ++k) row[k] = v[k];
      } else {
        const int pi = tl.pt_begin + lp;
        const size_t b = 9 * (size_t)nc + 3 * (size_t)pi;
        g[b] = (S)v[0];
        g[b + 1] = (S)v[1];
        g[b + 2] = (S)v[2];
        double* H = Hpp + 6 * (size_t)pi;
#pragma unroll
        for (int k = 0; k < 6; ++k) H[k] = v[3 + k];
        D[b] = (S)clamp_diag(v[3]);
        D[b + 1] = (S)clamp_diag(v[6]);
        D[b + 2] = (S)clamp_diag(v[8]);
      }
    }
  };
  // Two tiles per iteration, both tiles' loads issued before either is
  // computed.  Lanes past a tile's end, and a second tile past the range,
  // read clamped in-range addresses; their values are unused.
  for (int t = blockIdx.x * 4 + wv; t < n_tiles; t += 2 * stride) {
    const int t2 = t + stride;
    const Tile ta = tiles[t], tb = tiles[min(t2, n_tiles - 1)];
    const int na = tile_nobs(ta.info), nb = t2 < n_tiles ? tile_nobs(tb.info) : 0;
    const int oa = ta.obs_begin + min(lane, na - 1);
    const int ob = tb.obs_begin + min(lane, max(nb, 1) - 1);
    const uint32_t ma = meta[oa], mb = meta[ob];
    // every load of both tiles first (camera rows in the working precision,
    // float32 ones gathered by quads of lanes: these gathers bound the
    // kernel); the barrier keeps the first tile's conversions from waiting on
    // its loads before the second tile's are issued
    CamReq<S> rqa, rqb;
    cam_request<S>(camtab, (int)(ma & ((1u << kCamBits) - 1)), rqa);
    cam_request<S>(camtab, (int)(mb & ((1u << kCamBits) - 1)), rqb);
    S xa[3], xb[3];
    load_point<S>(pts, (size_t)(ta.pt_begin + (int)(ma >> kCamBits)), xa);
    load_point<S>(pts, (size_t)(tb.pt_begin + (int)(mb >> kCamBits)), xb);
    const P2 qa = reinterpret_cast<const P2*>(px)[oa];
    const P2 qb = reinterpret_cast<const P2*>(px)[ob];
    __builtin_amdgcn_sched_barrier(0);
    const Cam<S> ca = cam_take<S>(rqa), cb = cam_take<S>(rqb);
    tile(ta, na, ma, ca, xa, qa, oa);
    if (t2 < n_tiles) tile(tb, nb, mb, cb, xb, qb, ob);
  }
  const double tot = block_sum(cost, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kPartialWidth] = tot;
}

// Point side of the linearisation with recomputed blocks, one lane per lane
// unit (a point, or a piece of at most kLaneObsMax observations of a point
// with more): the lane loops over its observations (the tile's trip count),
// evaluates residual and blocks, and keeps g_p and the upper triangle of H_p
// in registers; whole points write their rows directly, pieces a split row
// that k_lin_split adds up.  The camera row and pixel of the next
// observation are requested before the current one is evaluated, from a
// meta word requested one step earlier still.  (With stored blocks the
// observation-per-lane kernel k_lin_points writes them coalesced instead.)
template <typename S>
__global__ __launch_bounds__(256) void k_lin_lanes(int n_tiles, const int2* __restrict__ ltiles, int n_units,
                                                   const int* __restrict__ unit_obs, const int* __restrict__ unit_pt,
                                                   const int* __restrict__ unit_row, const uint32_t* __restrict__ meta,
                                                   const S* __restrict__ px, const S* __restrict__ camtab,
                                                   const S* __restrict__ pts, S* __restrict__ g, S* __restrict__ D,
                                                   double* __restrict__ Hpp, double* __restrict__ split_rows, int nc,
                                                   double* __restrict__ partials, int loss, double loss_c,
                                                   S* __restrict__ wts) {
  __shared__ double red[4];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t cmask = (1u << kCamBits) - 1u;
  using P2 = typename Pair<S>::type;
  double cost = 0.0;
  for (int t = blockIdx.x * 4 + wv; t < n_tiles; t += gridDim.x * 4) {
    const int trip = ltiles[t].x;
    const int u = t * kWave + lane;
    const bool valid = u < n_units;
    const int uc = valid ? u : n_units - 1;
    const int ob = unit_obs[uc];
    const int k = valid ? unit_obs[uc + 1] - ob : 0;
    const unsigned ptw = (unsigned)unit_pt[uc];
    const int pt = (int)(ptw & 0x3fffffffu);
    // observation of step i (any of the unit's when the lane has none left).
    // In this order the lanes of a step share cameras (each point's camera
    // list is sorted, hot cameras first), which the camera-row gathers
    // profit from; the product rotates the order instead, to spread its LDS
    // atomics (a build that used the product's order here, to share its
    // step-ordered meta words, measured 2% slower in float32 and 12% in
    // float64).
    auto obs = [&](int i) { return i < k ? ob + i : ob; };
    S Xp[3];
    load_point<S>(pts, (size_t)pt, Xp);
    double v[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) v[a] = 0.0;
    CamReq<S> rq;
    cam_request<S>(camtab, (int)(meta[ob] & cmask), rq);
    P2 q = reinterpret_cast<const P2*>(px)[ob];
    uint32_t m1 = meta[obs(1)];
    for (int it = 0; it < trip; ++it) {
      const bool act = it < k;
      const int o = obs(it);
      // this observation's camera (every lane: float32 rows come by quads)
      const Cam<S> c = cam_take<S>(rq);
      // requests: the next observation's camera row and pixel, the meta word
      // of the one after
      cam_request<S>(camtab, (int)(m1 & cmask), rq);
      const P2 qn = reinterpret_cast<const P2*>(px)[obs(it + 1)];
      const uint32_t m2 = meta[obs(it + 2)];
      if (act) {
        S r0, r1, col[12][2];
        snavely_jacobian<S>(c, Xp[0], Xp[1], Xp[2], (S)q.x, (S)q.y, r0, r1, col);
        if (loss == CASPAR_LOSS_TRIVIAL) {
          cost = fma((double)r0, (double)r0, fma((double)r1, (double)r1, cost));
        } else {
          // robust loss: cost rho(s); residual and blocks scaled by sqrt(rho'(s))
          double w;
          cost += robust_rho(loss, loss_c, fma((double)r0, (double)r0, (double)r1 * (double)r1), w);
          const S sw = (S)sqrt(w);
          r0 *= sw;
          r1 *= sw;
#pragma unroll
          for (int j = 9; j < 12; ++j) {
            col[j][0] *= sw;
            col[j][1] *= sw;
          }
          wts[o] = (S)w;
        }
        double jp[3][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          jp[a][0] = col[9 + a][0];
          jp[a][1] = col[9 + a][1];
          v[a] = fma(jp[a][0], (double)r0, fma(jp[a][1], (double)r1, v[a]));
        }
        v[3] = fma(jp[0][0], jp[0][0], fma(jp[0][1], jp[0][1], v[3]));
        v[4] = fma(jp[0][0], jp[1][0], fma(jp[0][1], jp[1][1], v[4]));
        v[5] = fma(jp[0][0], jp[2][0], fma(jp[0][1], jp[2][1], v[5]));
        v[6] = fma(jp[1][0], jp[1][0], fma(jp[1][1], jp[1][1], v[6]));
        v[7] = fma(jp[1][0], jp[2][0], fma(jp[1][1], jp[2][1], v[7]));
        v[8] = fma(jp[2][0], jp[2][0], fma(jp[2][1], jp[2][1], v[8]));
      }
      q = qn;
      m1 = m2;
    }
    if (valid) {
      if ((ptw >> 31) != 0u) {
        double* row = split_rows + (size_t)unit_row[u] * kPtRowWidth;
#pragma unroll
        for (int a = 0; a < 9; ++a) row[a] = v[a];
      } else {
        const size_t b = 9 * (size_t)nc + 3 * (size_t)pt;
        g[b] = (S)v[0];
        g[b + 1] = (S)v[1];
        g[b + 2] = (S)v[2];
        double* H = Hpp + 6 * (size_t)pt;
#pragma unroll
        for (int a = 0; a < 6; ++a) H[a] = v[3 + a];
        D[b] = (S)clamp_diag(v[3]);
        D[b + 1] = (S)clamp_diag(v[6]);
        D[b + 2] = (S)clamp_diag(v[8]);
      }
    }
  }
  const double tot = block_sum(cost, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kPartialWidth] = tot;
}

// Points cut into pieces: sum their pieces' rows.
template <typename S>
__global__ void k_lin_split(int n_split, const SplitPoint* __restrict__ sp,
                            const double* __restrict__ split_rows, S* g, S* D, double* Hpp, int nc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_split) return;
  const SplitPoint s = sp[i];
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = 0; r < s.nrows; ++r)
    for (int k = 0; k < 9; ++k) v[k] += split_rows[(size_t)(s.row_begin + r) * kPtRowWidth + k];
  const size_t b = 9 * (size_t)nc + 3 * (size_t)s.pt;
  for (int k = 0; k < 3; ++k) g[b + k] = (S)v[k];
  for (int k = 0; k < 6; ++k) Hpp[6 * (size_t)s.pt + k] = v[3 + k];
  D[b] = (S)clamp_diag(v[3]);
  D[b + 1] = (S)clamp_diag(v[6]);
  D[b + 2] = (S)clamp_diag(v[8]);
}

// Points without observations: g = 0, H = 0, D at its floor.
template <typename S>
__global__ void k_lin_orphans(int n_orphan, S* g, S* D, double* Hpp, int nc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_orphan) return;
  const size_t b = 9 * (size_t)nc + 3 * (size_t)i;
  for (int k = 0; k < 3; ++k) {
    g[b + k] = (S)0;
    D[b + k] = (S)1e-6;
  }
  for (int k = 0; k < 6; ++k) Hpp[6 * (size_t)i + k] = 0.0;
}

// ---------------------------------------------------------------------------
// Camera-major block sums: one workgroup per chunk.
// ---------------------------------------------------------------------------

// One butterfly step of a wave reduce-scatter over N (even) values: lanes
// with bit M clear keep the sums of values [0, N/2), lanes with it set those
// of [N/2, N), both in positions [0, N/2).
template <int N, int M>
__device__ inline void scatter_step(double* v, int lane) {
  constexpr int H = N / 2;
  const bool up = (lane & M) != 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = up ? v[i] : v[i + H];
    const double keep = up ? v[i + H] : v[i];
    v[i] = keep + __shfl_xor(send, M, kWave);
  }
}

// Wave sums of the kCamRowWidth (54) values in v, one per lane: returns the
// index of the sum this lane holds in v[0], or -1.  Six butterfly steps move
// 27 + 14 + 7 + 4 + 2 + 1 values per lane instead of six per value; the
// halves of odd length are padded with a zero.
__device__ inline int wave_scatter54(double* v, int lane) {
  static_assert(kCamRowWidth == 54, "reduce-scatter is laid out for 54 values");
  scatter_step<54, 32>(v, lane);
  v[27] = 0.0;
  scatter_step<28, 16>(v, lane);
  scatter_step<14, 8>(v, lane);
  v[7] = 0.0;
  scatter_step<8, 4>(v, lane);
  scatter_step<4, 2>(v, lane);
  scatter_step<2, 1>(v, lane);
  const int pos3 = (lane & 4) + (lane & 2) + (lane & 1);           // of 7 (+ pad)
  const int pos1 = ((lane & 16) ? 14 : 0) + ((lane & 8) ? 7 : 0) + pos3;  // of 27 (+ pad)
  if (pos3 >= 7 || pos1 >= 27) return -1;
  return ((lane & 32) ? 27 : 0) + pos1;
}

// Workgroups [0, n_big) take chunk blockIdx.x with all four waves: thread t
// takes the chunk's observations t, t + 256, ...  Later workgroups take four
// small chunks, one per wave: lane l takes observations l, l + 64, ...  In
// both, a thread holds at most kPer observations, whose point indices,
// points and pixels are all requested before the first block is evaluated.
template <typename S>
__global__ __launch_bounds__(256) void k_lin_cams(const Chunk* __restrict__ chunks, int n_big, int n_chunks,
                                                  const int* __restrict__ cm_pt,
                                                  const S* __restrict__ cm_px,
                                                  const double* __restrict__ cam,
                                                  const S* __restrict__ pts,
                                                  double* __restrict__ rows, int loss, double loss_c) {
  constexpr int kPer = kCamChunk / 256;
  static_assert(kCamSmallChunk <= kPer * kWave, "a small chunk fits one wave");
  __shared__ double lds[4][kCamRowWidth];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const bool packed = (int)blockIdx.x >= n_big;  // workgroup-uniform
  const int ci = packed ? n_big + 4 * ((int)blockIdx.x - n_big) + wv : (int)blockIdx.x;
  if (packed && ci >= n_chunks) return;  // a wave without a chunk (last workgroup only)
  const Chunk ch = chunks[ci];
  const int me = packed ? lane : tid;
  const int step = packed ? kWave : 256;
  using P2 = typename Pair<S>::type;
  const Cam<S> c = load_cam<S>(cam, ch.cam);
  // A thread's own sums run over at most kPer observations in the working
  // precision: in the float32-mixed form, whose Jacobian and residual
  // entries are float32 already, the rounding of eight float32 products
  // stays far below that of the entries themselves, and the float32 sums
  // take half the registers (more waves in flight for the gathers).  Every
  // sum across threads (the wave reduce-scatter, the workgroup, the chunk
  // rows) is float64.
  S part[kCamRowWidth];
#pragma unroll
  for (int k = 0; k < kCamRowWidth; ++k) part[k] = (S)0;
  // float64 operands take twice the registers: two rounds of four
  constexpr int kAhead = sizeof(S) == 4 ? kPer : kPer / 2;
#pragma unroll
  for (int h = 0; h < kPer; h += kAhead) {
    int jj[kAhead];
    S xp[kAhead][3];
    P2 q[kAhead];
#pragma unroll
    for (int i = 0; i < kAhead; ++i) jj[i] = cm_pt[min(ch.begin + me + step * (h + i), ch.end - 1)];
#pragma unroll
    for (int i = 0; i < kAhead; ++i) {
      load_point<S>(pts, (size_t)jj[i], xp[i]);
      q[i] = reinterpret_cast<const P2*>(cm_px)[min(ch.begin + me + step * (h + i), ch.end - 1)];
    }
#pragma unroll
    for (int i = 0; i < kAhead; ++i) {
      if (ch.begin + me + step * (h + i) >= ch.end) break;
      S r0, r1, col[12][2];
      snavely_jacobian<S>(c, xp[i][0], xp[i][1], xp[i][2], (S)q[i].x, (S)q[i].y, r0, r1, col);
      if (loss != CASPAR_LOSS_TRIVIAL) {
        // the same weight as the point side computes for this observation
        double w;
        (void)robust_rho(loss, loss_c, fma((double)r0, (double)r0, (double)r1 * (double)r1), w);
        const S sw = (S)sqrt(w);
        r0 *= sw;
        r1 *= sw;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
          col[j][0] *= sw;
          col[j][1] *= sw;
        }
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) part[k] = fma(col[k][0], r0, fma(col[k][1], r1, part[k]));
#pragma unroll
      for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int l = k; l < 9; ++l)
          part[9 + tri9(k, l)] = fma(col[k][0], col[l][0], fma(col[k][1], col[l][1], part[9 + tri9(k, l)]));
    }
  }
  double acc[kCamRowWidth];
#pragma unroll
  for (int k = 0; k < kCamRowWidth; ++k) acc[k] = (double)part[k];
  const int idx = wave_scatter54(acc, lane);
  if (packed) {
    if (idx >= 0) rows[(size_t)ch.row * kCamRowWidth + idx] = acc[0];
    return;
  }
  if (idx >= 0) lds[wv][idx] = acc[0];
  __syncthreads();
  if (tid < kCamRowWidth) {
    const double s = lds[0][tid] + lds[1][tid] + lds[2][tid] + lds[3][tid];
    rows[(size_t)ch.row * kCamRowWidth + tid] = s;
  }
}

// Per camera (one workgroup): sum the chunk rows into g_c, H_cc and D_c.
// Lane k of each of the 16 waves takes value k (k < 54) of every 16th chunk
// with four independent accumulators, so each wave reads whole 432-byte
// rows and the most observed camera (over a thousand chunks) keeps 64 rows
// in flight; the 16 wave sums are added in LDS.
constexpr int kCamFinalWaves = 16;

template <typename S>
__global__ __launch_bounds__(kCamFinalWaves * 64) void k_lin_cam_final(int nc, const int* __restrict__ chunk_off,
                                                                        const double* __restrict__ rows, S* g, S* D,
                                                                        double* Hcc) {
  constexpr int W = kCamFinalWaves;
  __shared__ double red[W][kCamRowWidth];
  const int c = blockIdx.x;
  const int k = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int q0 = chunk_off[c], q1 = chunk_off[c + 1];
  if (k < kCamRowWidth) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = q0 + wv;
    for (; q + 3 * W < q1; q += 4 * W) {
      s0 += rows[(size_t)q * kCamRowWidth + k];
      s1 += rows[(size_t)(q + W) * kCamRowWidth + k];
      s2 += rows[(size_t)(q + 2 * W) * kCamRowWidth + k];
      s3 += rows[(size_t)(q + 3 * W) * kCamRowWidth + k];
    }
    for (; q < q1; q += W) s0 += rows[(size_t)q * kCamRowWidth + k];
    red[wv][k] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
  if (threadIdx.x < kCamRowWidth) {
    const int t = threadIdx.x;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < W; ++i) s += red[i][t];
    if (t < 9) {
      g[9 * (size_t)c + t] = (S)s;
    } else {
      const int hidx = t - 9;
      Hcc[45 * (size_t)c + hidx] = s;
      for (int d = 0; d < 9; ++d)
        if (tri9(d, d) == hidx) D[9 * (size_t)c + d] = (S)clamp_diag(s);
    }
  }
}

// Sum of column `col` of the first n partial slots into scal->red[slot].
__global__ void k_sum_partials(int n, const double* __restrict__ partials, int col, DevScalars* sc,
                               int slot) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[(size_t)i * kPartialWidth + col];
  s = block_sum(s, red);
  if (threadIdx.x == 0) sc->red[slot] = s;
}

// ---------------------------------------------------------------------------
// Cost only (trial step, float64 re-evaluation).
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_cost(int n_tiles, const Tile* __restrict__ tiles,
                                              const uint32_t* __restrict__ meta,
                                              const S* __restrict__ px,
                                              const S* __restrict__ camtab,
                                              const double* __restrict__ X,
                                              double* __restrict__ partials, int loss, double loss_c) {
  __shared__ double red[4];
  const int lane = threadIdx.x & (kWave - 1);
  // wave-uniform tile index: descriptors come through the scalar cache
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int stride = gridDim.x * 4;
  double cost = 0.0;
  // Two tiles per iteration, both tiles' loads issued before either is
  // computed.  Lanes past a tile's end, and a second tile past the range,
  // read clamped in-range addresses; their values are unused.
  for (int t = blockIdx.x * 4 + wv; t < n_tiles; t += 2 * stride) {
    const int t2 = t + stride;
    const Tile ta = tiles[t], tb = tiles[min(t2, n_tiles - 1)];
    const int na = tile_nobs(ta.info), nb = t2 < n_tiles ? tile_nobs(tb.info) : 0;
    const int oa = ta.obs_begin + min(lane, na - 1);
    const int ob = tb.obs_begin + min(lane, max(nb, 1) - 1);
    const uint32_t ma = meta[oa], mb = meta[ob];
    // every load of both tiles first (camera rows in the working precision,
    // float32 ones gathered by quads of lanes: these gathers bound the
    // kernel); the barrier keeps the first tile's conversions from waiting on
    // its loads before the second tile's are issued
    CamReq<S> rqa, rqb;
    cam_request<S>(camtab, (int)(ma & ((1u << kCamBits) - 1)), rqa);
    cam_request<S>(camtab, (int)(mb & ((1u << kCamBits) - 1)), rqb);
    const double* Xa = X + 3 * (size_t)(ta.pt_begin + (int)(ma >> kCamBits));
    const double* Xb = X + 3 * (size_t)(tb.pt_begin + (int)(mb >> kCamBits));
    const double xa[3] = {Xa[0], Xa[1], Xa[2]}, xb[3] = {Xb[0], Xb[1], Xb[2]};
    using P2 = typename Pair<S>::type;
    const P2 qa = reinterpret_cast<const P2*>(px)[oa];
    const P2 qb = reinterpret_cast<const P2*>(px)[ob];
    __builtin_amdgcn_sched_barrier(0);
    const Cam<S> ca = cam_take<S>(rqa), cb = cam_take<S>(rqb);
    // rho(|r|^2) of one observation (|r|^2 with the trivial loss)
    auto term = [&](S r0, S r1) {
      const double sq = fma((double)r0, (double)r0, (double)r1 * (double)r1);
      double w;
      return loss == CASPAR_LOSS_TRIVIAL ? sq : robust_rho(loss, loss_c, sq, w);
    };
    S r0, r1;
    snavely_residual<S>(ca, (S)xa[0], (S)xa[1], (S)xa[2], (S)qa.x, (S)qa.y, r0, r1);
    if (lane < na) cost += term(r0, r1);
    snavely_residual<S>(cb, (S)xb[0], (S)xb[1], (S)xb[2], (S)qb.x, (S)qb.y, r0, r1);
    if (lane < nb) cost += term(r0, r1);
  }
  const double tot = block_sum(cost, red);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kPartialWidth] = tot;
}

// ---------------------------------------------------------------------------
// Retraction: R Exp(dw), t + dt, calibration + d, X + dX (Section V).
// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_retract_cams(int nc, const double* __restrict__ cam, const S* __restrict__ delta,
                               double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double* in = cam + (size_t)c * kCamStride;
  const S* d = delta + 9 * (size_t)c;
  double E[9], R[9];
  so3_exp((double)d[0], (double)d[1], (double)d[2], E);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      R[3 * i + j] = in[3 * i] * E[j] + in[3 * i + 1] * E[3 + j] + in[3 * i + 2] * E[6 + j];
  double* o = out + (size_t)c * kCamStride;
  for (int i = 0; i < 9; ++i) o[i] = R[i];
  for (int i = 0; i < 6; ++i) o[9 + i] = in[9 + i] + (double)d[3 + i];
  o[15] = 0.0;
}

template <typename S>
__global__ void k_retract_points(int np, const double* __restrict__ X, const S* __restrict__ delta,
                                 double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < 3 * (int64_t)np) out[i] = X[i] + (double)delta[i];
}

// ---------------------------------------------------------------------------
// Parity hook: residuals and Jacobian blocks in caller order, float64.
// ---------------------------------------------------------------------------
template <typename S, bool RJ>
__global__ void k_export_lin(int n_tiles, const Tile* __restrict__ tiles, const uint32_t* __restrict__ meta,
                             const double* __restrict__ px, const double* __restrict__ cam,
                             const double* __restrict__ X, const void* J, const S* __restrict__ cam_s,
                             const S* __restrict__ wts, const int* __restrict__ s2c, double* resid, double* jc,
                             double* jp) {
  const int t = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (t >= n_tiles) return;
  const Tile tl = tiles[t];
  if (lane >= tile_nobs(tl.info)) return;
  const int o = tl.obs_begin + lane;
  const uint32_t m = meta[o];
  const int ci = (int)(m & ((1u << kCamBits) - 1));
  const int pi = tl.pt_begin + (int)(m >> kCamBits);
  const size_t c = (size_t)s2c[o];
  // robust loss: the sqrt(w)-scaled residual and blocks (stored blocks are
  // stored scaled already)
  const double sw = wts ? sqrt((double)wts[o]) : 1.0;
  if (resid) {
    const Cam<S> cm = load_cam<S>(cam, ci);
    const double* Xp = X + 3 * (size_t)pi;
    const double2 q = reinterpret_cast<const double2*>(px)[o];
    S r0, r1;
    snavely_residual<S>(cm, (S)Xp[0], (S)Xp[1], (S)Xp[2], (S)q.x, (S)q.y, r0, r1);
    resid[2 * c] = wts ? (double)(r0 * (S)sw) : (double)r0;
    resid[2 * c + 1] = wts ? (double)(r1 * (S)sw) : (double)r1;
  }
  S col[12][2];
  jacobian_of<S, RJ>(J, cam_s, X, o, ci, pi, col);
  if (RJ && wts)
    for (int j = 0; j < 12; ++j) {
      col[j][0] *= (S)sw;
      col[j][1] *= (S)sw;
    }
  if (jc)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 9; ++j) jc[18 * c + 9 * i + j] = col[j][i];
  if (jp)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j) jp[6 * c + 3 * i + j] = col[9 + j][i];
}

// ---------------------------------------------------------------------------
// Host drivers.
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int threads) {
  return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads);
}

// Workgroups of a 4-wave tile-walking kernel: as many as are resident on the
// chip at once (a second, partly filled round would leave CUs idle), within
// the partial-sum slots and the tiles.
template <auto Kern>
static unsigned tile_grid(int n_tiles) {
  static const int per_cu = [] {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(Kern), 256, 0) != hipSuccess)
      b = 1;
    return std::max(b, 1);
  }();
  return (unsigned)std::max(1, std::min({(n_tiles + 3) / 4, per_cu * kNumCUs, kMaxPartials}));
}

template <typename S>
static void linearize_t(caspar_ba* h) {
  hipStream_t st = h->stream;
  S* g = (S*)h->vec.g;
  S* D = (S*)h->vec.D;
  const unsigned tg = h->rj ? tile_grid<k_lin_lanes<S>>(h->n_lane_tiles) : tile_grid<k_lin_points<S, true>>(h->n_tiles);
  // camera rows in the working precision (float32 rows feed the point side
  // and the products; float64 reads the master rows unless the products
  // recompute their blocks)
  const bool cast = sizeof(S) == 4 || h->rj;
  if (cast && h->nc > 0) {
    k_cam_cast<S><<<nblk((int64_t)h->nc * kCamStride, 256), 256, 0, st>>>(h->nc * kCamStride, h->cam,
                                                                          (S*)h->cam_s);
    CBA_LAUNCHED();
  }
  if (h->rj && h->nc > 0) {
    k_cam_quat<S><<<nblk(h->nc, 256), 256, 0, st>>>(h->nc, h->cam, (S*)h->p_cam);
    CBA_LAUNCHED();
  }
  const S* camtab = cast ? (const S*)h->cam_s : (const S*)h->cam;
  if (sizeof(S) == 4 && h->np > 0) {
    k_point_cast<<<nblk(h->np, 256), 256, 0, st>>>(h->np, h->X, (float4*)h->pts_s);
    CBA_LAUNCHED();
  }
  const S* ptab = (const S*)pts_table(h);
  if (h->rj ? h->n_lane_tiles > 0 : h->n_tiles > 0) {
    if (h->rj)
    {
      k_lin_lanes<S><<<tg, 256, 0, st>>>(h->n_lane_tiles, h->lane_tiles, h->n_units, h->unit_obs, h->unit_pt,
                                         h->unit_row, h->meta, pixels_of<S>(h), camtab, ptab, g, D, h->Hpp,
                                         h->lane_split_rows, h->nc, h->partials, h->loss, h->loss_c, (S*)h->wts);
      CBA_LAUNCHED();
      // the product reads the IRLS weights in its step order
      if (h->loss != CASPAR_LOSS_TRIVIAL) launch_lane_weights(h);
    } else
      k_lin_points<S, true><<<tg, 256, 0, st>>>(h->n_tiles, h->tiles, h->meta, pixels_of<S>(h), camtab, ptab, h->J, g, D,
                                                h->Hpp, h->split_rows, h->nc, h->partials, h->loss, h->loss_c,
                                                (S*)h->wts);
    CBA_LAUNCHED();
    k_sum_partials<<<1, 1024, 0, st>>>((int)tg, h->partials, 0, h->scal, 0);
    CBA_LAUNCHED();
  } else {
    CBA_HIP(hipMemsetAsync(h->scal->red, 0, sizeof(double), st));
  }
  const int n_split = h->rj ? h->n_lane_split_pts : h->n_split_pts;
  if (n_split > 0) {
    k_lin_split<S><<<nblk(n_split, 256), 256, 0, st>>>(n_split, h->rj ? h->lane_split_pts : h->split_pts,
                                                       h->rj ? h->lane_split_rows : h->split_rows, g, D, h->Hpp,
                                                       h->nc);
    CBA_LAUNCHED();
  }
  if (h->n_orphan_pts > 0) {
    k_lin_orphans<S><<<nblk(h->n_orphan_pts, 256), 256, 0, st>>>(h->n_orphan_pts, g, D, h->Hpp, h->nc);
    CBA_LAUNCHED();
  }
  if (h->n_chunks > 0) {
    const int n_small = h->n_chunks - h->n_big_chunks;
    k_lin_cams<S><<<h->n_big_chunks + (n_small + 3) / 4, 256, 0, st>>>(
        h->chunks, h->n_big_chunks, h->n_chunks, h->cm_pt, cm_pixels_of<S>(h), h->cam, ptab, h->chunk_rows, h->loss,
        h->loss_c);
    CBA_LAUNCHED();
  }
  if (h->nc > 0) {
    k_lin_cam_final<S><<<h->nc, kCamFinalWaves * 64, 0, st>>>(h->nc, h->chunk_off, h->chunk_rows, g, D, h->Hcc);
    CBA_LAUNCHED();
  }
  run_between_lin(h);  // pose between-factors: their g, H_cc, D terms and cost
}

void run_linearize(caspar_ba* h) {
  if (h->prec == CASPAR_FP64)
    linearize_t<double>(h);
  else
    linearize_t<float>(h);
  launch_absmax(h, h->vec.g);  // read back with the cost sums
  const DevScalars s = read_scalars(h);
  h->cost = 0.5 * (s.red[0] + (h->n_between > 0 ? s.red[7] : 0.0));
  h->gmax = h->N > 0 ? s.red[3] : 0.0;
  h->linearized = true;
  h->bj_lambda = -1.0;
}

double run_cost(caspar_ba* h, const double* cam, const double* X, bool fp64) {
  launch_cost(h, cam, X, fp64);
  return cost_of(h, read_scalars(h));
}

double cost_of(const caspar_ba* h, const DevScalars& s) {
  return 0.5 * (s.red[1] + (h->n_between > 0 ? s.red[7] : 0.0));
}

// Reprojection cost sum into red[1] (zero without observations) and the
// between-factor sum into red[7].
void launch_cost(caspar_ba* h, const double* cam, const double* X, bool fp64) {
  launch_between_cost(h, cam);  // pose between-factors (float64)
  if (h->n_tiles == 0) {
    k_sum_partials<<<1, 1024, 0, h->stream>>>(0, h->partials, 0, h->scal, 1);
    CBA_LAUNCHED();
    return;
  }
  hipStream_t st = h->stream;
  const bool f64 = fp64 || h->prec == CASPAR_FP64;
  const unsigned tg = f64 ? tile_grid<k_cost<double>>(h->n_tiles) : tile_grid<k_cost<float>>(h->n_tiles);
  if (f64) {
    k_cost<double><<<tg, 256, 0, st>>>(h->n_tiles, h->tiles, h->meta, pixels_of<double>(h), cam, X, h->partials, h->loss,
                                       h->loss_c);
  } else {
    // float32 rows of the cameras being evaluated, so the residual kernel
    // gathers 64 bytes per observation instead of 128
    k_cam_cast<float><<<nblk((int64_t)h->nc * kCamStride, 256), 256, 0, st>>>(h->nc * kCamStride, cam,
                                                                              (float*)h->cam_trial_s);
    CBA_LAUNCHED();
    k_cost<float><<<tg, 256, 0, st>>>(h->n_tiles, h->tiles, h->meta, pixels_of<float>(h), (const float*)h->cam_trial_s, X,
                                      h->partials, h->loss, h->loss_c);
  }
  CBA_LAUNCHED();
  k_sum_partials<<<1, 1024, 0, st>>>((int)tg, h->partials, 0, h->scal, 1);
  CBA_LAUNCHED();
}

template <typename S>
static void retract_t(caspar_ba* h, const S* delta) {
  hipStream_t st = h->stream;
  if (h->nc) {
    k_retract_cams<S><<<nblk(h->nc, 256), 256, 0, st>>>(h->nc, h->cam, delta, h->cam_trial);
    CBA_LAUNCHED();
  }
  if (h->np) {
    k_retract_points<S><<<nblk(3 * (int64_t)h->np, 256), 256, 0, st>>>(h->np, h->X, delta + 9 * (size_t)h->nc,
                                                                       h->X_trial);
    CBA_LAUNCHED();
  }
}

void run_retract(caspar_ba* h, const void* delta) {
  if (h->prec == CASPAR_FP64)
    retract_t<double>(h, (const double*)delta);
  else
    retract_t<float>(h, (const float*)delta);
}

void run_export_linearization(caspar_ba* h, double* resid, double* jc, double* jp) {
  if (h->n_tiles == 0) return;
  const unsigned grid = nblk((int64_t)h->n_tiles * kWave, 256);
#define CBA_EXPORT(S, RJ)                                                                                 \
  k_export_lin<S, RJ><<<grid, 256, 0, h->stream>>>(h->n_tiles, h->tiles, h->meta, h->px, h->cam, h->X, h->J, \
                                                   (const S*)h->cam_s, weights_of<S>(h), h->obs_s2c, resid, jc, jp)
  if (h->prec == CASPAR_FP64) {
    if (h->rj)
      CBA_EXPORT(double, true);
    else
      CBA_EXPORT(double, false);
  } else {
    if (h->rj)
      CBA_EXPORT(float, true);
    else
      CBA_EXPORT(float, false);
  }
#undef CBA_EXPORT
  CBA_LAUNCHED();
}

}  // namespace cba
