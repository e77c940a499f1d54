// Fused damped normal-equation product w = (J^T J + lambda D) p and
// p^T w = |J p|^2 + lambda p^T D p, matrix-free (Section V: the normal
// equations are solved directly; J^T J is never formed).
//
// Per observation o with camera c and point j:  q_o = J_c,o p_c + J_j,o p_j,
// camera contribution J_c,o^T q_o (9), point contribution J_j,o^T q_o (3).
//
// The paper's shared-add accessor (Section IV-A) reduces per block and then
// issues one global atomic per unique index.  On MI355X global FP64 atomics
// sustain only ~22 G/s, far below the rate observations stream in, so these
// kernels keep all camera accumulation on chip instead:
//  * persistent workgroups each own a contiguous range of wave tiles and keep
//    float64 accumulators for the K most observed cameras (and a window of
//    cold ones) in LDS (ds_add_f64), flushed once per workgroup as plain rows;
//  * observations of the remaining cameras write their 9-vector to a row of
//    their own (ballot-ranked inside the wave, so rows stay coalesced);
//  * stored blocks (k_matvec): one observation per lane; points are
//    contiguous inside a tile, so an in-wave segmented scan sums their
//    contributions and the first lane of each point writes w_j directly;
//  * recomputed blocks (k_matvec_lanes): one point per lane, looping over its
//    observations with the point sum in registers.
// A second small kernel adds the per-workgroup rows and cold rows of each
// camera in a fixed order, handles split and orphan points and turns the
// p^T A p partials into alpha for PCG.  The LDS sums themselves are atomic
// adds in the order the waves happen to reach them, so the camera side of w
// (and with it every later PCG iterate) varies from run to run at the
// rounding level; the point side and the fixed-order second pass do not.
#include <hip/hip_ext.h>

#include <mutex>

#include "common.hpp"
#include "model.hpp"

namespace cba {

// Camera part of p copied into the 16-byte aligned camera rows the product
// gathers (row_stride values per camera, p at row_off, zeros to the row's
// end).
template <typename S>
__global__ void k_pad_cams(int nc, const S* __restrict__ p, S* __restrict__ out, int row_stride, int row_off,
                           const DevScalars* __restrict__ sc) {
  if (sc != nullptr && sc->done) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  S* o = out + (size_t)c * row_stride + row_off;
  for (int k = 0; k < row_stride - row_off; ++k) o[k] = k < 9 ? p[9 * (size_t)c + k] : (S)0;
}

template <typename S>
__device__ inline void load_cam_row(const S* __restrict__ rows, int c, S* out);
template <>
__device__ inline void load_cam_row<double>(const double* __restrict__ rows, int c, double* out) {
  const double2* r = reinterpret_cast<const double2*>(rows + (size_t)c * CamPad<double>::n);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const double2 v = r[i];
    out[2 * i] = v.x;
    out[2 * i + 1] = v.y;
  }
}
// float32 rows (64 bytes) come in two halves, as camera rows do in the
// linearisation: requested by quads of lanes, then exchanged within the quad
// (both with every lane active).
template <typename S>
struct CamRowReq;
template <>
struct CamRowReq<float> {
  QuadRows r;
};
template <>
struct CamRowReq<double> {
  double v[CamPad<double>::n];
};
__device__ inline void cam_row_request(const float* __restrict__ rows, int c, CamRowReq<float>& q) {
  static_assert(CamPad<float>::n == 16, "64-byte float32 rows");
  quad_rows_request(rows, c, q.r);
}
__device__ inline void cam_row_request(const double* __restrict__ rows, int c, CamRowReq<double>& q) {
  load_cam_row<double>(rows, c, q.v);
}
__device__ inline void cam_row_take(CamRowReq<float>& q, float (&out)[CamPad<float>::n]) { quad_rows_take(q.r, out); }
__device__ inline void cam_row_take(CamRowReq<double>& q, double (&out)[CamPad<double>::n]) {
#pragma unroll
  for (int k = 0; k < CamPad<double>::n; ++k) out[k] = q.v[k];
}

// Launch shape of the fused product (RJ: recomputed blocks, the
// point-per-lane kernel) and pipeline depth of the stored-block kernel.  16
// waves per workgroup; the float64 point-per-lane kernel needs more than 128
// VGPRs, so it runs 8-wave workgroups (256 VGPRs per lane).  One tile ahead of
// the one being computed, the stored-block kernel requests
//   prefetch_j:   the stored Jacobian chunks (float32: 24 VGPRs; float64 has
//                 no room and loads them at the end of the previous tile);
//   prefetch_pt:  p and D of the tile's points (otherwise loaded with the
//                 camera gathers of the tile itself);
//   prefetch_cam: the camera rows of p (otherwise gathered at the start of
//                 the tile, with their latency exposed; float64 would spill).
template <typename S, bool RJ>
struct MvCfg {
  static constexpr int threads = 1024;
  static constexpr bool prefetch_j = true;
  static constexpr bool prefetch_pt = true;
  static constexpr bool prefetch_cam = true;
};
template <>
struct MvCfg<double, false> {
  static constexpr int threads = 1024;
  static constexpr bool prefetch_j = false;
  static constexpr bool prefetch_pt = true;
  static constexpr bool prefetch_cam = false;
};
template <>
struct MvCfg<double, true> {
  static constexpr int threads = 512;
};

int matvec_waves(int prec, bool rj) {
  if (prec == CASPAR_FP64) return (rj ? MvCfg<double, true>::threads : MvCfg<double, false>::threads) / kWave;
  return (rj ? MvCfg<float, true>::threads : MvCfg<float, false>::threads) / kWave;
}

// Workgroup size of the point-per-lane product on a problem too small to
// give every CU a workgroup of the full size: four waves.
constexpr int kLanesSmallThreads = 256;
int matvec_small_waves() { return kLanesSmallThreads / kWave; }

// Stores that only some lanes need are issued by every lane through a buffer
// resource: a lane with nothing to write passes an offset past the end of
// the buffer and the hardware drops its write.  Each loop iteration then
// issues the same memory operations on every path, so the compiler's wait
// counts stay exact and no load waits for a store issued after it.
constexpr unsigned kDropOffset = 0x80000000u;

__device__ inline __amdgpu_buffer_rsrc_t buffer_of(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

using u32x4 = unsigned __attribute__((ext_vector_type(4)));
using u32x3 = unsigned __attribute__((ext_vector_type(3)));
using u32x2 = unsigned __attribute__((ext_vector_type(2)));

// One cold row at byte offset off: 9 values, padded to ColdRow<S>::n in
// float64 (five 16-byte stores); in float32 two 16-byte stores and one
// 4-byte store (rows 4-byte aligned).
__device__ inline void store_cold_row(__amdgpu_buffer_rsrc_t rs, unsigned off, const double v[9]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const double2 d = make_double2(v[2 * i], i < 4 ? v[2 * i + 1] : 0.0);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, d), rs, (int)off + 16 * i, 0, 0);
  }
}

__device__ inline void store_cold_row(__amdgpu_buffer_rsrc_t rs, unsigned off, const float v[9]) {
  static_assert(ColdRow<float>::n == 9, "float32 cold rows are 9 values");
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const u32x4 u = {__float_as_uint(v[4 * i]), __float_as_uint(v[4 * i + 1]), __float_as_uint(v[4 * i + 2]),
                     __float_as_uint(v[4 * i + 3])};
    __builtin_amdgcn_raw_buffer_store_b128(u, rs, (int)off + 16 * i, 0, 0);
  }
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[8]), rs, (int)off + 32, 0, 0);
}

// Three consecutive scalars at byte offset off.
__device__ inline void store3(__amdgpu_buffer_rsrc_t rs, unsigned off, const float v[3]) {
  const u32x3 u = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2])};
  __builtin_amdgcn_raw_buffer_store_b96(u, rs, (int)off, 0, 0);
}
__device__ inline void store3(__amdgpu_buffer_rsrc_t rs, unsigned off, const double v[3]) {
  const double2 d = make_double2(v[0], v[1]);
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, d), rs, (int)off, 0, 0);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v[2]), rs, (int)off + 16, 0, 0);
}

template <typename S>
__global__ __launch_bounds__((MvCfg<S, false>::threads)) void k_matvec(
    int n_tiles, int G, const Tile* __restrict__ tiles, const uint32_t* __restrict__ meta,
    const void* __restrict__ J, const S* __restrict__ pts_s,
    const S* __restrict__ p_cam, const int* __restrict__ cold_lo,
    const S* __restrict__ p, const S* __restrict__ D, double lambda, S* __restrict__ w, int nc, int K,
    int n_orphan, S* __restrict__ hot_rows, S* __restrict__ cold_rows, double* __restrict__ win_rows,
    double* __restrict__ split_rows,
    double* __restrict__ partials, DevScalars* __restrict__ sc, int P, int L, int local_base,
    unsigned w_pt_bytes, unsigned cold_bytes) {
  constexpr int THREADS = MvCfg<S, false>::threads;
  constexpr int WAVES = THREADS / kWave;
  constexpr bool PREFETCH_J = MvCfg<S, false>::prefetch_j;
  constexpr bool PF_PT = MvCfg<S, false>::prefetch_pt;
  constexpr bool PF_CAM = MvCfg<S, false>::prefetch_cam;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* hot = reinterpret_cast<double*>(lds_raw);        // [K][9] camera sums
  // the P most observed cameras get kPrivCopies private copies (copy = lane
  // mod kPrivCopies), so lanes of one wave hitting the same camera mostly
  // update different addresses; folded into hot[] before the flush
  double* priv = hot + (size_t)K * 9;                      // [kPrivCopies][P][9]
  // this workgroup's window of cold cameras [lo, lo + L)
  double* win = priv + (size_t)kPrivCopies * P * 9;        // [L][9]
  const int lo = L > 0 ? cold_lo[blockIdx.x] : 0;
  __shared__ double red[WAVES];
  if (sc != nullptr && sc->done) {
    // the iteration after the one that stopped PCG: its x step has been taken
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->last_x = 0;
    return;
  }
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  for (int i = tid; i < (K + kPrivCopies * P + L) * 9; i += THREADS) hot[i] = 0.0;
  __syncthreads();

  const S* __restrict__ pp_base = p + 9 * (size_t)nc;
  const S* __restrict__ dp_base = D + 9 * (size_t)nc;
  S* __restrict__ wp_base = w + 9 * (size_t)nc;
  const __amdgpu_buffer_rsrc_t w_rs = buffer_of(wp_base, w_pt_bytes);
  const __amdgpu_buffer_rsrc_t cold_rs = buffer_of(cold_rows, cold_bytes);
  double pap = 0.0;
  const int t0 = (int)((int64_t)n_tiles * blockIdx.x / G);
  const int t1 = (int)((int64_t)n_tiles * (blockIdx.x + 1) / G);

  // Software pipeline over the wave's tiles t, t + W, t + 2W, t + 3W (W =
  // waves per workgroup):
  //   tile t       being computed: meta word, Jacobian columns, p and D of
  //                its points and the camera rows of p are in registers
  //                (whatever the configuration does not prefetch is
  //                gathered at the start of the tile);
  //   tile t + W   meta in registers; its Jacobian columns, point data and
  //                camera rows are requested during tile t;
  //   tile t + 2W  meta requested during tile t;
  //   tile t + 3W  descriptor requested during tile t.
  // The tile index is wave-uniform, so descriptors come through the scalar
  // cache.  Every vector load is issued unconditionally (lanes past a tile's
  // end, and tiles past the range, read clamped in-range addresses and
  // their values are unused), so each iteration issues a fixed number of
  // loads and every wait covers exactly the loads it needs.
  int t = t0 + __builtin_amdgcn_readfirstlane(wv);
  if (t < t1) {
    auto nobs = [&](int ti, const Tile& T) { return ti < t1 ? tile_nobs(T.info) : 0; };
    auto olane = [&](int k) { return min(lane, max(k, 1) - 1); };
    auto tile_at = [&](int ti) { return tiles[min(ti, t1 - 1)]; };
    // Registers of one tile.  The loop is unrolled by two over a pair of
    // these, so the set being computed and the set being filled swap roles
    // instead of being copied.
    struct Regs {
      S col[12][2];         // Jacobian columns
      S pjv[3], dpv[3];     // p and D of the observation's point
      CamRowReq<S> pcr;     // camera row of p, as requested
    };
    // the requests made one tile ahead (tile descriptor T, nt observations,
    // meta word mm of this lane)
    auto request = [&](Regs& R, const Tile& T, int nt, uint32_t mm) {
      // (blocks are stored sqrt(w)-scaled under a robust loss)
      if (PREFETCH_J) JStore<S>::load(J, T.obs_begin + olane(nt), R.col);
      if (PF_PT) {
        const size_t b = 3 * (size_t)(T.pt_begin + (int)(mm >> kCamBits));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          R.pjv[k] = pp_base[b + k];
          R.dpv[k] = dp_base[b + k];
        }
      }
      if (PF_CAM) cam_row_request(p_cam, (int)(mm & ((1u << kCamBits) - 1)), R.pcr);
    };
    Tile tl = tiles[t], tln = tile_at(t + WAVES), tlnn = tile_at(t + 2 * WAVES);
    int n = tile_nobs(tl.info);
    uint32_t m = meta[tl.obs_begin + olane(n)];
    uint32_t mn = meta[tln.obs_begin + olane(nobs(t + WAVES, tln))];
    Regs A, B;
    request(A, tl, n, m);
    if (!PREFETCH_J) JStore<S>::load(J, tl.obs_begin + olane(n), A.col);

    // One tile: compute tile t from cur while the next tile's data comes
    // into nxt.  Returns true after the wave's last tile.
    auto step = [&](Regs& cur, Regs& nxt) -> bool {
      const bool act = lane < n;
      const int ci_raw = (int)(m & ((1u << kCamBits) - 1));
      const int lp_raw = (int)(m >> kCamBits);
      const int ci = act ? ci_raw : -1;
      const int lp = act ? lp_raw : 100 + lane;
      // 1. gathers of the current tile that the configuration does not
      //    prefetch
      if (!PF_CAM) cam_row_request(p_cam, ci_raw, cur.pcr);
      // the camera row of p, taken by every lane (float32 rows come by quads)
      // before the next tile's requests claim their registers
      S pcv[CamPad<S>::n];
      cam_row_take(cur.pcr, pcv);
      if (!PF_PT) {
        const size_t b = 3 * (size_t)(tl.pt_begin + lp_raw);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          cur.pjv[k] = pp_base[b + k];
          cur.dpv[k] = dp_base[b + k];
        }
      }
      // 2. requests for the next tiles, issued after the gathers so that
      //    waiting for the gathers does not wait for them
      __builtin_amdgcn_sched_barrier(0);
      const int tn = t + WAVES;
      request(nxt, tln, nobs(tn, tln), mn);
      const uint32_t mnn = meta[tlnn.obs_begin + olane(nobs(tn + WAVES, tlnn))];
      const Tile tl3 = tile_at(tn + 2 * WAVES);
      __builtin_amdgcn_sched_barrier(0);
      // 3. the current tile
      S yc[9], yp[3];
#pragma unroll
      for (int k = 0; k < 9; ++k) yc[k] = (S)0;
#pragma unroll
      for (int k = 0; k < 3; ++k) yp[k] = (S)0;
      if (act) {
        const S(&col)[12][2] = cur.col;
        S q0 = (S)0, q1 = (S)0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          q0 = fma(col[k][0], pcv[k], q0);
          q1 = fma(col[k][1], pcv[k], q1);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          q0 = fma(col[9 + k][0], cur.pjv[k], q0);
          q1 = fma(col[9 + k][1], cur.pjv[k], q1);
        }
        pap = fma((double)q0, (double)q0, fma((double)q1, (double)q1, pap));
#pragma unroll
        for (int k = 0; k < 9; ++k) yc[k] = fma(col[k][0], q0, col[k][1] * q1);
#pragma unroll
        for (int k = 0; k < 3; ++k) yp[k] = fma(col[9 + k][0], q0, col[9 + k][1] * q1);
        // LDS sums: the most observed cameras into their private copies,
        // the other hot cameras, and the cold cameras of this workgroup's
        // window
        const unsigned slot = (unsigned)(ci - lo);
        if (ci < K || slot < (unsigned)L) {
          double* a = ci < P ? priv + ((size_t)(lane % kPrivCopies) * P + ci) * 9
                             : (ci < K ? hot + 9 * ci : win + 9 * slot);
#pragma unroll
          for (int k = 0; k < 9; ++k) atomicAdd(a + k, (double)yc[k]);
        }
      }
      // cold cameras outside the window: each such observation writes its
      // own row, numbered from the tile's cold_begin in lane order
      const bool scat = act && ci >= K && (unsigned)(ci - lo) >= (unsigned)L;
      const unsigned long long sm = __ballot(scat);
      {
        const unsigned row = (unsigned)tl.cold_begin + (unsigned)__popcll(sm & ((1ull << lane) - 1ull));
        store_cold_row(cold_rs, scat ? row * (unsigned)(ColdRow<S>::n * sizeof(S)) : kDropOffset, yc);
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
      const bool split = tile_split(tl.info);
      // lambda p^T D p, once per point
      if (head && (!split || tile_first(tl.info))) {
        S dpp = (S)0;
#pragma unroll
        for (int k = 0; k < 3; ++k) dpp = fma(cur.dpv[k] * cur.pjv[k], cur.pjv[k], dpp);
        pap = fma(lambda, (double)dpp, pap);
      }
      // the point rows of w (ordinary tiles)
      {
        S wv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) wv[k] = fma((S)lambda * cur.dpv[k], cur.pjv[k], yp[k]);
        const unsigned off = (unsigned)(3 * (tl.pt_begin + lp)) * (unsigned)sizeof(S);
        store3(w_rs, head && !split ? off : kDropOffset, wv);
      }
      // a slice of a point with more than kTileMax observations: its row
      if (split && head) {
        double* row = split_rows + (size_t)tl.split_row * kPtRowWidth;
#pragma unroll
        for (int k = 0; k < 3; ++k) row[k] = (double)yp[k];
      }
      // 4. advance
      t = tn;
      if (t >= t1) return true;
      tl = tln;
      n = nobs(t, tl);
      m = mn;
      tln = tlnn;
      mn = mnn;
      tlnn = tl3;
      if (!PREFETCH_J) JStore<S>::load(J, tl.obs_begin + olane(n), nxt.col);
      return false;
    };
    for (;;) {
      if (step(A, B)) break;
      if (step(B, A)) break;
    }
  }
  // lambda p^T D p of the camera blocks and of points without observations
  for (int i = blockIdx.x * THREADS + tid; i < 9 * nc; i += G * THREADS) {
    const double v = p[i];
    pap = fma(lambda * (double)D[i] * v, v, pap);
  }
  for (int i = blockIdx.x * THREADS + tid; i < 3 * n_orphan; i += G * THREADS) {
    const double v = pp_base[i];
    pap = fma(lambda * (double)dp_base[i] * v, v, pap);
  }
  const double tot = block_sum(pap, red);  // (also orders the LDS updates before the fold)
  if (tid == 0) partials[(size_t)blockIdx.x * kPartialWidth] = tot;
  for (int i = tid; i < P * 9; i += THREADS) {
    double s = hot[i];
#pragma unroll
    for (int c = 0; c < kPrivCopies; ++c) s += priv[(size_t)c * P * 9 + i];
    hot[i] = s;
  }
  __syncthreads();
  // the workgroup's hot-camera sums, rounded to the working precision (the
  // products are float32 in the mixed form; the sum over workgroups is float64)
  S* dst = hot_rows + (size_t)blockIdx.x * K * 9;
  for (int i = tid; i < K * 9; i += THREADS) dst[i] = (S)hot[i];
  double* wdst = win_rows + (size_t)blockIdx.x * L * kColdRow;
  for (int i = tid; i < L * 9; i += THREADS) wdst[(size_t)(i / 9) * kColdRow + i % 9] = win[i];
}

// Point-per-lane fused product (recomputed blocks).  A wave tile is 64
// consecutive lane units: a point with at most kLaneObsMax observations, or a
// piece of one with more.  Lane l takes unit 64 t + l, loads its point's X,
// p and D once, and loops over the unit's observations (trip count: the
// tile's largest unit), keeping the point sum J_p^T q in registers; the
// observation of iteration i is (i + l) mod k (an order fixed at create, see
// the step-ordered tables below): neighbouring lanes take
// different ranks of their points' camera lists (each sorted by camera),
// so the lanes of one LDS access that hit the same camera (the most observed
// one, or the tile's shared least observed one) are spread over the wave.  Camera sums go to LDS
// (hot cameras, the window) or to cold rows exactly as in k_matvec, the rows
// numbered per tile in (iteration, lane) order.  A whole point writes its row
// of w directly (64 consecutive points per tile: coalesced); a piece writes a
// split row that k_matvec_final adds up.  The meta words come from a copy in
// this step order (built at create), so the 64 reads of a step are one
// coalesced request instead of 64 gathers.  W: a robust loss's IRLS weights,
// which come in the same step order (copied there after each linearisation).
template <typename S, int THREADS, bool W>
__global__ __launch_bounds__(THREADS) void k_matvec_lanes(
    int n_tiles, int G, const int2* __restrict__ ltiles, int n_units, const int* __restrict__ unit_obs,
    const int* __restrict__ unit_pt, const int* __restrict__ unit_row, const int* __restrict__ lbase,
    const uint32_t* __restrict__ lmeta, const S* __restrict__ pts_s, const S* __restrict__ p_cam,
    const int* __restrict__ cold_lo,
    const S* __restrict__ p, const S* __restrict__ D, double lambda, S* __restrict__ w, int nc, int K,
    int n_orphan, S* __restrict__ hot_rows, S* __restrict__ cold_rows, double* __restrict__ win_rows,
    double* __restrict__ split_rows, double* __restrict__ partials, DevScalars* __restrict__ sc, int P, int L,
    unsigned w_pt_bytes, unsigned cold_bytes, const S* __restrict__ lwts) {
  constexpr int WAVES = THREADS / kWave;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* hot = reinterpret_cast<double*>(lds_raw);        // [K][9] camera sums
  double* priv = hot + (size_t)K * 9;                      // [kPrivCopies][P][9]
  double* win = priv + (size_t)kPrivCopies * P * 9;        // [L][9]
  const int lo = L > 0 ? cold_lo[blockIdx.x] : 0;
  __shared__ double red[WAVES];
  if (sc != nullptr && sc->done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->last_x = 0;
    return;
  }
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  for (int i = tid; i < (K + kPrivCopies * P + L) * 9; i += THREADS) hot[i] = 0.0;
  __syncthreads();

  const S* __restrict__ pp_base = p + 9 * (size_t)nc;
  const S* __restrict__ dp_base = D + 9 * (size_t)nc;
  S* __restrict__ wp_base = w + 9 * (size_t)nc;
  const __amdgpu_buffer_rsrc_t w_rs = buffer_of(wp_base, w_pt_bytes);
  const __amdgpu_buffer_rsrc_t cold_rs = buffer_of(cold_rows, cold_bytes);
  const uint32_t cmask = (1u << kCamBits) - 1u;
  double pap = 0.0;
  const int t0 = (int)((int64_t)n_tiles * blockIdx.x / G);
  const int t1 = (int)((int64_t)n_tiles * (blockIdx.x + 1) / G);

  // Software pipeline over the wave's steps (tile t, iteration i), tiles
  // t, t + W, t + 2W, ... (W waves), every tile at least two iterations long:
  //   step s         computed: its camera row (and IRLS weight) in registers;
  //   step s + 1     camera row requested during step s, from its meta word;
  //   step s + 2     meta word requested during step s.
  // Steps s + 1 and s + 2 lie in the current tile or the next one, so the
  // unit data (first observation, count, point) are kept for this tile and the
  // next two, and the point data (X, p, D) for this tile and the next.
  int t = t0 + __builtin_amdgcn_readfirstlane(wv);
  if (t < t1) {
    // (the observation a lane visits at a step is fixed at create: the meta
    // words and IRLS weights come in step order, so the kernel needs only the
    // unit's observation count)
    struct Unit {
      int k;
      unsigned ptw;
    };
    // lanes of a tile past the range (or past the last unit) get k = 0 and
    // in-range addresses
    auto unit_at = [&](int tt) {
      Unit U;
      const int u = tt * kWave + lane;
      const bool valid = tt < t1 && u < n_units;
      const int uc = valid ? u : n_units - 1;
      U.k = valid ? unit_obs[uc + 1] - unit_obs[uc] : 0;
      U.ptw = valid ? (unsigned)unit_pt[uc] : 0u;
      return U;
    };
    struct Pt {
      S x[3], p[3], d[3];
    };
    auto point_of = [&](const Unit& U) {
      Pt P;
      const int pt = (int)(U.ptw & 0x3fffffffu);
      load_point<S>(pts_s, (size_t)pt, P.x);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        P.p[q] = pp_base[3 * (size_t)pt + q];
        P.d[q] = dp_base[3 * (size_t)pt + q];
      }
      return P;
    };
    auto tile_info = [&](int tt) { return ltiles[min(tt, n_tiles - 1)]; };
    // first step of a tile in the step-ordered meta words (tiles past the
    // last read the last one's first steps; their lanes have k = 0)
    auto base_of = [&](int tt) { return lbase[min(tt, n_tiles - 1)]; };
    auto meta_at = [&](int b, int i) { return lmeta[((size_t)b + i) * kWave + lane]; };
    auto wgt_at = [&](int b, int i) { return lwts[((size_t)b + i) * kWave + lane]; };

    Unit Uc = unit_at(t), Un = unit_at(t + WAVES), Unn = unit_at(t + 2 * WAVES);
    int2 ti_c = tile_info(t), ti_n = tile_info(t + WAVES);
    Pt Pc = point_of(Uc), Pn = point_of(Un);
    int it = 0;
    int cold_row = ti_c.y;
    S acc[3] = {(S)0, (S)0, (S)0};
    // step s (current), s + 1 and their observations; meta of s + 1
    int b_c = base_of(t), b_n = base_of(t + WAVES);
    uint32_t m_1 = meta_at(b_c, 1);  // trip >= 2
    struct Row {
      S c[kProdCamRow];
      S wgt;
      int cid;  // the camera
    };
    Row RA, RB;
    {
      const uint32_t m0 = meta_at(b_c, 0);
      load_prod_cam<S>(p_cam, (int)(m0 & cmask), RA.c);
      if constexpr (W) RA.wgt = wgt_at(b_c, 0);
      RA.cid = (int)(m0 & cmask);
    }

    // One step: compute step s from cur while step s + 1's row comes into
    // nxt.  Returns true after the wave's last step.
    auto step = [&](Row& cur, Row& nxt) -> bool {
      // the next step and the one after: this tile or the next
      const bool in_tile1 = it + 1 < ti_c.x, in_tile2 = it + 2 < ti_c.x;
      __builtin_amdgcn_sched_barrier(0);
      // requests: the row of step s + 1, the meta word of step s + 2
      load_prod_cam<S>(p_cam, (int)(m_1 & cmask), nxt.c);
      if constexpr (W) nxt.wgt = wgt_at(in_tile1 ? b_c : b_n, in_tile1 ? it + 1 : 0);
      nxt.cid = (int)(m_1 & cmask);
      const uint32_t m_2 = meta_at(in_tile2 ? b_c : b_n, in_tile2 ? it + 2 : it + 2 - ti_c.x);
      __builtin_amdgcn_sched_barrier(0);
      // step s
      const bool act = it < Uc.k;
      const int ci_raw = cur.cid;
      S yc[9], yp[3];
#pragma unroll
      for (int q = 0; q < 9; ++q) yc[q] = (S)0;
      const int ci = act ? ci_raw : -1;
      if (act) {
        const Cam<S> cam = prod_cam<S>(cur.c);
        const S* pc = cur.c + kProdCamP;
        const S qwq = snavely_apply<W, S>(cam, Pc.x[0], Pc.x[1], Pc.x[2], pc, Pc.p, W ? cur.wgt : (S)1, yc, yp);
        pap += (double)qwq;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] += yp[q];
        const unsigned slot = (unsigned)(ci - lo);
        if (ci < K || slot < (unsigned)L) {
          double* a = ci < P ? priv + ((size_t)(lane % kPrivCopies) * P + ci) * 9
                             : (ci < K ? hot + 9 * ci : win + 9 * slot);
#pragma unroll
          for (int q = 0; q < 9; ++q) atomicAdd(a + q, (double)yc[q]);
        }
      }
      // cold cameras outside the window: rows in (iteration, lane) order
      const bool scat = act && ci >= K && (unsigned)(ci - lo) >= (unsigned)L;
      const unsigned long long sm = __ballot(scat);
      {
        const unsigned row = (unsigned)cold_row + (unsigned)__popcll(sm & ((1ull << lane) - 1ull));
        store_cold_row(cold_rs, scat ? row * (unsigned)(ColdRow<S>::n * sizeof(S)) : kDropOffset, yc);
      }
      cold_row += (int)__popcll(sm);
      // advance
      m_1 = m_2;
      if (++it < ti_c.x) return false;
      // end of the tile: the point's row of w (whole points) or its split row
      {
        const bool valid = Uc.k > 0;
        const bool piece = (Uc.ptw >> 31) != 0u;
        const bool first = ((Uc.ptw >> 30) & 1u) != 0u;
        const int pt = (int)(Uc.ptw & 0x3fffffffu);
        S dpp = (S)0;
#pragma unroll
        for (int q = 0; q < 3; ++q) dpp = fma(Pc.d[q] * Pc.p[q], Pc.p[q], dpp);
        if (valid && (!piece || first)) pap = fma(lambda, (double)dpp, pap);
        if (valid && piece) {
          double* row = split_rows + (size_t)unit_row[t * kWave + lane] * kPtRowWidth;
#pragma unroll
          for (int q = 0; q < 3; ++q) row[q] = (double)acc[q];
        }
        S wv3[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) wv3[q] = fma((S)lambda * Pc.d[q], Pc.p[q], acc[q]);
        store3(w_rs, valid && !piece ? (unsigned)(3 * pt) * (unsigned)sizeof(S) : kDropOffset, wv3);
      }
      t += WAVES;
      if (t >= t1) return true;
      it = 0;
      Uc = Un;
      Un = Unn;
      Unn = unit_at(t + 2 * WAVES);
      Pc = Pn;
      Pn = point_of(Un);
      ti_c = ti_n;
      ti_n = tile_info(t + WAVES);
      b_c = b_n;
      b_n = base_of(t + WAVES);
      cold_row = ti_c.y;
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[q] = (S)0;
      return false;
    };
    for (;;) {
      if (step(RA, RB)) break;
      if (step(RB, RA)) break;
    }
  }
  // lambda p^T D p of the camera blocks and of points without observations
  for (int i = blockIdx.x * THREADS + tid; i < 9 * nc; i += G * THREADS) {
    const double v = p[i];
    pap = fma(lambda * (double)D[i] * v, v, pap);
  }
  for (int i = blockIdx.x * THREADS + tid; i < 3 * n_orphan; i += G * THREADS) {
    const double v = pp_base[i];
    pap = fma(lambda * (double)dp_base[i] * v, v, pap);
  }
  const double tot = block_sum(pap, red);  // (also orders the LDS updates before the fold)
  if (tid == 0) partials[(size_t)blockIdx.x * kPartialWidth] = tot;
  for (int i = tid; i < P * 9; i += THREADS) {
    double s2 = hot[i];
#pragma unroll
    for (int c = 0; c < kPrivCopies; ++c) s2 += priv[(size_t)c * P * 9 + i];
    hot[i] = s2;
  }
  __syncthreads();
  // the workgroup's hot-camera sums, rounded to the working precision (the
  // products are float32 in the mixed form; the sum over workgroups is float64)
  S* dst = hot_rows + (size_t)blockIdx.x * K * 9;
  for (int i = tid; i < K * 9; i += THREADS) dst[i] = (S)hot[i];
  double* wdst = win_rows + (size_t)blockIdx.x * L * kColdRow;
  for (int i = tid; i < L * 9; i += THREADS) wdst[(size_t)(i / 9) * kColdRow + i % 9] = win[i];
}

// Camera rows of w, split and orphan points, p^T A p and (in PCG) alpha.
// Block roles by index:
//   [0, nb_hot):           column sums of the per-workgroup rows of the LDS
//                          cameras (16 columns x 16 row groups per block);
//   [nb_hot, +nb_cold):    one wave per remaining camera, lanes striding its
//                          observation rows;
//   the rest:              split points and points without observations.
// Block 0 also turns the p^T A p partials into pAp (and alpha in PCG).
// hot-sum columns per final-kernel workgroup: one 128-byte line of each
// workgroup row, 256 threads = kHotCols columns x (256 / kHotCols) row groups
template <typename S>
constexpr int kHotCols = 128 / (int)sizeof(S);

template <typename S>
__global__ __launch_bounds__(256) void k_matvec_final(
    int nc, int K, int G, const S* __restrict__ hot_rows,
    const S* __restrict__ cold_rows, const double* __restrict__ win_rows, int local_base,
    const int* __restrict__ cold_off,
    const int* __restrict__ cold_list, const S* __restrict__ p, const S* __restrict__ D, double lambda,
    S* __restrict__ w, int n_split, const SplitPoint* __restrict__ sp, const double* __restrict__ split_rows,
    int n_orphan, const double* __restrict__ partials, DevScalars* __restrict__ sc, int pcg_mode, int nb_hot,
    int nb_cold, const double* __restrict__ bt_rows, int n_partials) {
  // between-factor part of camera entry i = 9 c + k (k < 6), if any
  auto between_part = [&](int64_t i) -> double {
    const int k = (int)(i % 9);
    return (bt_rows != nullptr && k < 6) ? bt_rows[(i / 9) * 6 + k] : 0.0;
  };
  __shared__ double red[4][64];
  if (pcg_mode && sc->done) return;
  const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
  const int b = blockIdx.x;
  if (b < nb_hot) {
    // HC consecutive columns (one 128-byte line per row) x RG row groups;
    // each thread sums every RG-th workgroup row with two independent
    // accumulators, then the RG group sums are added in LDS
    constexpr int HC = kHotCols<S>, RG = 256 / HC;
    double (*gsum)[HC] = reinterpret_cast<double (*)[HC]>(&red[0][0]);
    const int ncol = K * 9;
    const int cl = tid % HC, gr = tid / HC;
    const int col = b * HC + cl;
    double s0 = 0.0, s1 = 0.0;
    if (col < ncol) {
      const S* r = hot_rows + col;
      int g = gr;
      for (; g + RG < G; g += 2 * RG) {
        s0 += (double)r[(size_t)g * ncol];
        s1 += (double)r[(size_t)(g + RG) * ncol];
      }
      if (g < G) s0 += (double)r[(size_t)g * ncol];
    }
    gsum[gr][cl] = s0 + s1;
    __syncthreads();
    if (gr == 0 && col < ncol) {
      double tot = 0.0;
#pragma unroll
      for (int k = 0; k < RG; ++k) tot += gsum[k][cl];
      w[col] = (S)fma(lambda * (double)D[col], (double)p[col], tot + between_part(col));
    }
  } else if (b < nb_hot + nb_cold) {
    const int c = K + (b - nb_hot) * 4 + grp;
    if (c < nc) {
      const int q0 = cold_off[c - K], q1 = cold_off[c - K + 1];
      double acc[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) acc[k] = 0.0;
      for (int q = q0 + lane; q < q1; q += 64) {
        const int e = cold_list[q];
        if (e < local_base) {
          const S* row = cold_rows + (size_t)e * ColdRow<S>::n;
#pragma unroll
          for (int k = 0; k < 9; ++k) acc[k] += (double)row[k];
        } else {
          const double* row = win_rows + (size_t)(e - local_base) * kColdRow;
#pragma unroll
          for (int k = 0; k < 9; ++k) acc[k] += row[k];
        }
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const double tot = wave_sum(acc[k]);
        if (lane == 0) {
          const size_t i = 9 * (size_t)c + k;
          w[i] = (S)fma(lambda * (double)D[i], (double)p[i], tot + between_part((int64_t)i));
        }
      }
    }
  } else {
    const int64_t i = (int64_t)(b - nb_hot - nb_cold) * 256 + tid;
    const int64_t nsplit = 3 * (int64_t)n_split;
    if (i < nsplit) {
      const SplitPoint s = sp[i / 3];
      const int k = (int)(i % 3);
      double acc = 0.0;
      for (int r = 0; r < s.nrows; ++r) acc += split_rows[(size_t)(s.row_begin + r) * kPtRowWidth + k];
      const size_t bi = 9 * (size_t)nc + 3 * (size_t)s.pt + k;
      w[bi] = (S)fma(lambda * (double)D[bi], (double)p[bi], acc);
    } else if (i < nsplit + 3 * (int64_t)n_orphan) {
      const size_t bi = 9 * (size_t)nc + (size_t)(i - nsplit);
      w[bi] = (S)(lambda * (double)D[bi] * (double)p[bi]);
    }
  }
  if (b == 0) {
    double s = 0.0;
    for (int g = tid; g < n_partials; g += blockDim.x) s += partials[(size_t)g * kPartialWidth];
    s = block_sum(s, &red[0][0]);
    if (tid == 0) {
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

template <typename S, bool RJ>
static void launch_matvec(caspar_ba* h, double lambda, const S* p, S* w, DevScalars* scp) {
  constexpr int T_FULL = MvCfg<S, RJ>::threads;
  const int P = std::min(h->K, kPrivCams);
  const size_t lds = matvec_lds_bytes(h->K, h->L);
  auto kern = k_matvec<S>;
  // recomputed blocks run the point-per-lane kernel, in small workgroups on
  // a small problem, with IRLS weights under a robust loss
  const bool small = RJ && h->mv_small;
  const bool wtd = RJ && lane_weights_of<S>(h) != nullptr;
  constexpr int TL = MvCfg<S, true>::threads;
  auto lanes = small ? (wtd ? k_matvec_lanes<S, kLanesSmallThreads, true> : k_matvec_lanes<S, kLanesSmallThreads, false>)
                     : (wtd ? k_matvec_lanes<S, TL, true> : k_matvec_lanes<S, TL, false>);
  const int T = small ? kLanesSmallThreads : T_FULL;
  const void* kptr = RJ ? (const void*)lanes : (const void*)kern;
  // the dynamic-LDS limit belongs to the kernel on a device: raised only when
  // a launch needs more than it was last set to (not at every launch)
  {
    static std::mutex mu;
    static std::vector<size_t> lds_set[4];  // [full, small workgroups] x [unweighted, weighted]
    std::lock_guard<std::mutex> lock(mu);
    std::vector<size_t>& set = lds_set[(small ? 1 : 0) + (wtd ? 2 : 0)];
    if ((size_t)h->device >= set.size()) set.resize((size_t)h->device + 1, 65536);
    if (lds > set[h->device]) {
      CBA_HIP(hipFuncSetAttribute(kptr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      set[h->device] = lds;
    }
  }
  // with timing on, the launch itself stamps the events (no extra packets
  // between the kernels)
  hipEvent_t e0, e1;
  timing_events(h, &e0, &e1);
  if constexpr (RJ) {
    hipExtLaunchKernelGGL(lanes, dim3(h->G), dim3(T), (uint32_t)lds, h->stream, e0, e1, 0u,
                          h->n_lane_tiles, h->G, h->lane_tiles, h->n_units, h->unit_obs, h->unit_pt, h->unit_row,
                          h->lane_base, h->lane_meta, (const S*)pts_table(h), (const S*)h->p_cam, h->cold_lo, p,
                          (const S*)h->vec.D,
                          lambda, w, h->nc, h->K, h->n_orphan_pts, (S*)h->hot_rows, (S*)h->cold_rows,
                          h->win_rows, h->lane_split_rows, h->partials, scp, P, h->L,
                          (unsigned)(3 * (size_t)h->np * sizeof(S)),
                          (unsigned)((size_t)h->cold_local_base * ColdRow<S>::n * sizeof(S)), lane_weights_of<S>(h));
    CBA_LAUNCHED();
    return;
  }
  hipExtLaunchKernelGGL(kern, dim3(h->G), dim3(T), (uint32_t)lds, h->stream, e0, e1, 0u, h->n_tiles, h->G, h->tiles,
                        h->meta, h->J, (const S*)pts_table(h), (const S*)h->p_cam, h->cold_lo, p,
                        (const S*)h->vec.D, lambda, w, h->nc, h->K, h->n_orphan_pts, (S*)h->hot_rows,
                        (S*)h->cold_rows, h->win_rows, h->split_rows, h->partials, scp, P, h->L,
                        h->cold_local_base, (unsigned)(3 * (size_t)h->np * sizeof(S)),
                        (unsigned)((size_t)h->cold_local_base * ColdRow<S>::n * sizeof(S)));
  CBA_LAUNCHED();
}

template <typename S>
static void matvec_t(caspar_ba* h, double lambda, const S* p, S* w, bool pcg_mode, bool pad_cams) {
  hipStream_t st = h->stream;
  DevScalars* scp = pcg_mode ? h->scal : nullptr;
  if (h->n_tiles > 0 || h->nc > 0 || h->n_orphan_pts > 0) {
    if (pad_cams) {
      k_pad_cams<S><<<(unsigned)std::max(1, (h->nc + 255) / 256), 256, 0, st>>>(
          h->nc, p, (S*)h->p_cam, cam_row_stride<S>(h), cam_row_p_off(h), scp);
      CBA_LAUNCHED();
    }
    if (h->rj)
      launch_matvec<S, true>(h, lambda, p, w, scp);
    else
      launch_matvec<S, false>(h, lambda, p, w, scp);
  }
  // pose between-factors: their share of the camera rows and of p^T A p
  run_between_product(h, p, pcg_mode);
  const int n_partials = h->G + (h->n_between > 0 ? (int)between_grid(h) : 0);
  const int nb_hot = (h->K * 9 + kHotCols<S> - 1) / kHotCols<S>;
  const int nb_cold = (h->nc - h->K + 3) / 4;
  const int64_t nrest = 3 * (int64_t)(h->rj ? h->n_lane_split_pts : h->n_split_pts) + 3 * (int64_t)h->n_orphan_pts;
  const int nb_rest = (int)((nrest + 255) / 256);
  const unsigned grid = (unsigned)std::max(1, nb_hot + nb_cold + nb_rest);
  k_matvec_final<S><<<grid, 256, 0, st>>>(h->nc, h->K, h->G, (const S*)h->hot_rows,
                                          (const S*)h->cold_rows, h->win_rows, h->cold_local_base, h->cold_off,
                                          h->cold_list, p,
                                          (const S*)h->vec.D, lambda, w, h->rj ? h->n_lane_split_pts : h->n_split_pts,
                                          h->rj ? h->lane_split_pts : h->split_pts,
                                          h->rj ? h->lane_split_rows : h->split_rows, h->n_orphan_pts, h->partials,
                                          h->scal, pcg_mode ? 1 : 0,
                                          nb_hot, nb_cold, h->n_between > 0 ? h->bt_rows : nullptr, n_partials);
  CBA_LAUNCHED();
}

// The pair of HIP events that times the next launch of the fused product.
void timing_events(caspar_ba* h, hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (h->timing_every <= 0) return;
  const int pos = h->mv_in_solve++;
  if (h->mv_seq++ % h->timing_every != 0) return;
  if (h->ev_used == (int)h->ev_start.size()) {
    hipEvent_t a, b;
    CBA_HIP(hipEventCreate(&a));
    CBA_HIP(hipEventCreate(&b));
    h->ev_start.push_back(a);
    h->ev_stop.push_back(b);
    h->ev_pos.push_back(0);
  }
  h->ev_pos[h->ev_used] = pos;
  *start = h->ev_start[h->ev_used];
  *stop = h->ev_stop[h->ev_used];
  ++h->ev_used;
}

void timing_harvest(caspar_ba* h, int effective) {
  if (h->timing_every <= 0) return;
  for (int i = 0; i < h->ev_used; ++i) {
    if (h->ev_pos[i] >= effective) continue;  // the launch found the solve finished
    float ms = 0.f;
    CBA_HIP(hipEventSynchronize(h->ev_stop[i]));
    CBA_HIP(hipEventElapsedTime(&ms, h->ev_start[i], h->ev_stop[i]));
    h->mv_ms += ms;
    ++h->mv_launches;
  }
  h->ev_used = 0;
  h->mv_in_solve = 0;
}

void run_matvec(caspar_ba* h, double lambda, const void* p, void* w, bool pcg_mode, bool pad_cams) {
  if (h->prec == CASPAR_FP64)
    matvec_t<double>(h, lambda, (const double*)p, (double*)w, pcg_mode, pad_cams);
  else
    matvec_t<float>(h, lambda, (const float*)p, (float*)w, pcg_mode, pad_cams);
}

}  // namespace cba
