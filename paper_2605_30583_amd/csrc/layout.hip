// Problem set-up: arena planning, input validation, the observation ordering
// and index tables built once at create time, parameter and observation I/O,
// and the stand-alone projection.
//
// Ordering (built on the GPU with radix sorts, small tables on the host):
//  * cameras are relabelled by observation count, most observed first; the
//    first K of them are accumulated in LDS by the fused product;
//  * points are grouped by their least-observed camera (largest internal
//    camera id), so that observations of rarely seen cameras sit together;
//  * observations are sorted point-major (camera, then caller index, inside
//    a point) and cut into wave tiles of <= 64 observations holding whole
//    points (points seen more than 64 times get tiles of their own);
//  * a camera-major index over the same observations drives the per-camera
//    block sums.
// This is the role the paper's sorted block-unique index structure plays for
// its shared gather / scatter accessors (Section IV-A), laid out for 64-wide
// wavefronts.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.hpp"
#include "model.hpp"

namespace cba {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

void fail(int status, const std::string& msg) { throw Error{status, msg}; }

static size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

static int ceil_log2(long long v) {
  int b = 0;
  while ((1LL << b) < v) ++b;
  return b;
}

static size_t sort_temp_bytes(int64_t no) {
  size_t a = 0, b = 0;
  if (no > 0) {
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (const int*)nullptr, (int*)nullptr, (int)no, 0, 64) !=
            hipSuccess ||
        hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int*)nullptr, (int*)nullptr, (int)no, 0, 32) !=
            hipSuccess)
      return (size_t)-1;
  }
  return std::max(a, b) + (1 << 20);
}

static int groups_per_cu(int K, int L) { return matvec_lds_bytes(K, L) > 80 * 1024 ? 1 : 2; }

bool make_plan(int nc, int np, int64_t no, int mode, Plan& p) {
  if (nc < 0 || np < 0 || no < 0) return false;
  if (no >= (int64_t)1 << 31 || nc >= (1 << kCamBits)) return false;
  if ((mode & ~(1 | CASPAR_RECOMPUTE_JACOBIAN)) != 0) return false;
  const int prec = mode & 1;
  const bool rj = (mode & CASPAR_RECOMPUTE_JACOBIAN) != 0;
  if (no > 0 && (nc == 0 || np == 0)) return false;
  if (3 * (size_t)np * scalar_bytes(mode & 1) >= ((size_t)1 << 31)) return false;  // product's point rows
  if ((int64_t)9 * nc + 3 * (int64_t)np >= ((int64_t)1 << 31)) return false;
  const size_t s = scalar_bytes(prec);
  const size_t nch = prec == CASPAR_FP64 ? 12 : 6;
  const size_t sort_bytes = sort_temp_bytes(no);
  if (sort_bytes == (size_t)-1) return false;
  const size_t no_pad = align_up((size_t)no, kJBlock);
  const size_t N = 9 * (size_t)nc + 3 * (size_t)np;
  p = Plan{};
  p.K = std::min(nc, kMaxHot);
  p.G = groups_per_cu(p.K, std::min(kColdWin, nc - p.K)) * kNumCUs;
  p.max_tiles = (size_t)no / 16 + 8;
  p.max_chunks = (size_t)no / kCamChunk + nc + 1;
  p.max_cold = nc > p.K ? (size_t)((no * (int64_t)(nc - p.K)) / nc + 1) : 0;
  p.max_split_tiles = (size_t)no / 32 + 2;
  p.max_split_pts = (size_t)no / 65 + 1;
  // lane units: a point of k observations makes ceil(k / kLaneObsMax)
  p.max_units = (size_t)np + (size_t)no / kLaneObsMax + 1;
  p.max_lane_tiles = p.max_units / kWave + 1;
  p.max_pieces = (size_t)no / 8 + 2;
  p.max_lane_split_pts = (size_t)no / (kLaneObsMax + 1) + 1;

  size_t off = 0;
  auto take = [&](Plan::Region& r, size_t bytes) {
    r.off = off;
    r.bytes = bytes;
    off += align_up(bytes);
  };
  take(p.scal, sizeof(DevScalars));
  take(p.partials, (size_t)kMaxPartials * kPartialWidth * 8);
  take(p.gauge_rows, 256 * 35 * 8);
  take(p.cam, (size_t)nc * kCamStride * 8);
  take(p.cam_trial, (size_t)nc * kCamStride * 8);
  take(p.cam_s, (size_t)nc * kCamStride * s);
  take(p.cam_trial_s, (size_t)nc * kCamStride * 4);
  take(p.pts_s, prec == CASPAR_FP64 ? 16 : (size_t)np * 16);
  take(p.wts, (size_t)no * s + 16);
  take(p.X, (size_t)np * 3 * 8);
  take(p.X_trial, (size_t)np * 3 * 8);
  take(p.cam_c2i, (size_t)nc * 4);
  take(p.cam_i2c, (size_t)nc * 4);
  take(p.pt_c2i, (size_t)np * 4);
  take(p.pt_i2c, (size_t)np * 4);
  take(p.obs_s2c, (size_t)no * 4);
  take(p.meta, no_pad * 4);
  take(p.px, (size_t)no * 16);
  take(p.px_s, prec == CASPAR_FP64 ? 16 : (size_t)no * 8);
  // J doubles as the create-time scratch (sort buffers, counters).
  const size_t scratch = 2 * 8 * (size_t)no + 2 * 4 * (size_t)no + 4 * (size_t)no +
                         align_up(sort_bytes) + 8 * (size_t)np + 8 * (size_t)nc + 8192;
  take(p.J, std::max(rj ? 0 : nch * no_pad * 16, scratch));
  take(p.tiles, p.max_tiles * sizeof(Tile));
  take(p.cold_lo, (size_t)kMaxGroups * 4);
  take(p.p_cam, (size_t)nc * kProdCamRow * 8);
  take(p.cm_pt, (size_t)no * 4);
  take(p.cm_px, prec == CASPAR_FP64 ? (size_t)no * 16 : 16);
  take(p.cm_px_s, prec == CASPAR_FP64 ? 16 : (size_t)no * 8);
  take(p.cam_off, ((size_t)nc + 1) * 4);
  take(p.chunks, p.max_chunks * sizeof(Chunk));
  take(p.chunk_off, ((size_t)nc + 1) * 4);
  take(p.chunk_rows, p.max_chunks * kCamRowWidth * 8);
  const size_t max_cold_rows = nc > p.K ? p.max_cold + (size_t)kMaxGroups * kColdWin : 0;
  take(p.cold_list, max_cold_rows * 4 + 4);
  take(p.cold_off, ((size_t)(nc - p.K) + 1) * 4);
  // single-observation rows (ColdRow<S> each, at most max_cold of them), then
  // from the next 256-byte boundary the window rows (kColdRow doubles, at
  // most kMaxGroups * kColdWin of them)
  const size_t single_row_bytes = prec == CASPAR_FP64 ? ColdRow<double>::n * 8 : ColdRow<float>::n * 4;
  if (nc > p.K)
    take(p.cold_rows, align_up(p.max_cold * single_row_bytes) + (size_t)kMaxGroups * kColdWin * kColdRow * 8 + 256);
  else
    take(p.cold_rows, 256);
  take(p.split_pts, p.max_split_pts * sizeof(SplitPoint));
  take(p.split_rows, p.max_split_tiles * kPtRowWidth * 8);
  take(p.hot_rows, (size_t)p.G * p.K * 9 * scalar_bytes(prec));
  take(p.Hcc, (size_t)nc * 45 * 8);
  take(p.Hpp, (size_t)np * 6 * 8);
  take(p.Mc, (size_t)nc * 45 * s);
  take(p.Mp, (size_t)np * 6 * s);
  p.vec_bytes = align_up(std::max<size_t>(N, 1) * s);
  take(p.vecs, 8 * p.vec_bytes);
  take(p.cm_obs, (size_t)no * 4);
  take(p.unit_obs, (p.max_units + 1) * 4);
  take(p.unit_pt, p.max_units * 4 + 4);
  take(p.unit_row, p.max_units * 4 + 4);
  take(p.lane_tiles, p.max_lane_tiles * 8 + 8);
  take(p.lane_split_pts, p.max_lane_split_pts * sizeof(SplitPoint) + 16);
  take(p.lane_split_rows, p.max_pieces * kPtRowWidth * 8 + 8);
  // the point-per-lane kernels' meta words in their step order (recomputed
  // blocks; a lane tile has at most kLaneObsMax steps)
  take(p.lane_base, (p.max_lane_tiles + 1) * 4 + 4);
  take(p.lane_meta, rj ? p.max_lane_tiles * kWave * kLaneObsMax * 4 + 16 : 16);
  take(p.lane_wts, rj ? p.max_lane_tiles * kWave * kLaneObsMax * s + 16 : 16);
  p.total = off;
  return true;
}

// ---------------------------------------------------------------------------
// Kernels used at create time.
// ---------------------------------------------------------------------------
__global__ void k_validate(int nc, int np, int no, const double* __restrict__ cams,
                           const double* __restrict__ pts, const int* __restrict__ oc,
                           const int* __restrict__ op, const double* __restrict__ px,
                           DevScalars* sc) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int err = 0;
  if (i < no) {
    const int c = oc[i], p = op[i];
    if (c < 0 || c >= nc || p < 0 || p >= np) err |= 1;
    if (!isfinite(px[2 * i]) || !isfinite(px[2 * i + 1])) err |= 2;
  }
  if (i < (int64_t)nc * 9 && !isfinite(cams[i])) err |= 4;
  if (i < (int64_t)np * 3 && !isfinite(pts[i])) err |= 8;
  if (err) atomicOr(&sc->err, err);
}

// Observation counts per point (global atomics: a point has few
// observations, so they rarely collide) and, without the LDS histogram
// below, per camera too.
__global__ void k_count(int no, const int* __restrict__ oc, const int* __restrict__ op,
                        int* cam_cnt, int* pt_cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < no) {
    if (cam_cnt != nullptr) atomicAdd(&cam_cnt[oc[i]], 1);
    atomicAdd(&pt_cnt[op[i]], 1);
  }
}

// Observation counts per camera through a per-workgroup LDS histogram: the
// most observed cameras take millions of increments, which global atomics
// serialise at one address; each workgroup adds its bins once at the end.
constexpr int kCountLdsCams = 32768;  // 128 KiB of LDS
__global__ __launch_bounds__(1024) void k_count_cams(int no, const int* __restrict__ oc, int nc, int* cam_cnt) {
  extern __shared__ int hist[];
  for (int i = threadIdx.x; i < nc; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < no; o += gridDim.x * blockDim.x)
    atomicAdd(&hist[oc[o]], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < nc; i += blockDim.x)
    if (hist[i] != 0) atomicAdd(&cam_cnt[i], hist[i]);
}

__global__ void k_point_key(int no, const int* __restrict__ oc, const int* __restrict__ op,
                            const int* __restrict__ cam_c2i, int* pt_key) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < no) atomicMax(&pt_key[op[i]], cam_c2i[oc[i]]);
}

__global__ void k_make_keys(int no, const int* __restrict__ oc, const int* __restrict__ op,
                            const int* __restrict__ cam_c2i, const int* __restrict__ pt_c2i,
                            uint64_t* keys, int* vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < no) {
    keys[i] = ((uint64_t)(uint32_t)pt_c2i[op[i]] << kCamBits) | (uint64_t)(uint32_t)cam_c2i[oc[i]];
    vals[i] = i;
  }
}

// One wave per tile: meta word, sorted pixels, camera keys for the
// camera-major sort.
__global__ void k_fill_obs(int n_tiles, const Tile* __restrict__ tiles,
                           const uint64_t* __restrict__ skeys, const int* __restrict__ s2c,
                           const double* __restrict__ px_caller, uint32_t* meta, double* px,
                           uint32_t* cam_keys, int* cam_vals) {
  const int t = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (t >= n_tiles) return;
  const Tile tl = tiles[t];
  const int n = tile_nobs(tl.info);
  if (lane >= n) return;
  const int s = tl.obs_begin + lane;
  const uint64_t key = skeys[s];
  const int ci = (int)(key & ((1u << kCamBits) - 1));
  const int pi = (int)(key >> kCamBits);
  meta[s] = (uint32_t)ci | ((uint32_t)(pi - tl.pt_begin) << kCamBits);
  const int c = s2c[s];
  px[2 * s] = px_caller[2 * (size_t)c];
  px[2 * s + 1] = px_caller[2 * (size_t)c + 1];
  cam_keys[s] = (uint32_t)ci;
  cam_vals[s] = s;
}

// Camera-major point indices and observed pixels, the pixels in the working
// precision (the float32 kernels never read float64 camera-major pixels).
template <typename T>
__global__ void k_fill_cm(int no, const int* __restrict__ cm_obs, const uint64_t* __restrict__ skeys,
                          const double* __restrict__ px, int* cm_pt, T* cm_px) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < no) {
    const int s = cm_obs[j];
    cm_pt[j] = (int)(skeys[s] >> kCamBits);
    cm_px[2 * j] = (T)px[2 * s];
    cm_px[2 * j + 1] = (T)px[2 * s + 1];
  }
}




__global__ void k_cams_from_bal(int nc, const double* __restrict__ bal, const int* __restrict__ c2i,
                                double* cam) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double* b = bal + 9 * (size_t)c;
  double* o = cam + (size_t)c2i[c] * kCamStride;
  double R[9];
  so3_exp(b[0], b[1], b[2], R);
  for (int i = 0; i < 9; ++i) o[i] = R[i];
  for (int i = 0; i < 6; ++i) o[9 + i] = b[3 + i];
  o[15] = 0.0;
}

__global__ void k_cams_to_bal(int nc, const double* __restrict__ cam, const int* __restrict__ c2i,
                              double* bal) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double* in = cam + (size_t)c2i[c] * kCamStride;
  double R[9], w[3];
  for (int i = 0; i < 9; ++i) R[i] = in[i];
  so3_log(R, w);
  double* o = bal + 9 * (size_t)c;
  o[0] = w[0];
  o[1] = w[1];
  o[2] = w[2];
  for (int i = 0; i < 6; ++i) o[3 + i] = in[9 + i];
}

__global__ void k_points_in(int np, const double* __restrict__ in, const int* __restrict__ c2i,
                            double* X) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int q = c2i[p];
  for (int k = 0; k < 3; ++k) X[3 * (size_t)q + k] = in[3 * (size_t)p + k];
}

__global__ void k_points_out(int np, const double* __restrict__ X, const int* __restrict__ c2i,
                             double* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int q = c2i[p];
  for (int k = 0; k < 3; ++k) out[3 * (size_t)p + k] = X[3 * (size_t)q + k];
}

// float32 copies of both pixel orders (float32-mixed form).
__global__ void k_px_cast(int64_t n, const double2* __restrict__ a, float2* __restrict__ as) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 u = a[i];
    as[i] = make_float2((float)u.x, (float)u.y);
  }
}


__global__ void k_set_px(int no, const int* __restrict__ s2c, const double* __restrict__ px_caller,
                         double* px) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < no) {
    const size_t c = s2c[s];
    px[2 * s] = px_caller[2 * c];
    px[2 * s + 1] = px_caller[2 * c + 1];
  }
}

template <typename T>
__global__ void k_set_cm_px(int no, const int* __restrict__ cm_obs, const double* __restrict__ px, T* cm_px) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < no) {
    const int s = cm_obs[j];
    cm_px[2 * j] = (T)px[2 * s];
    cm_px[2 * j + 1] = (T)px[2 * s + 1];
  }
}

__global__ void k_project(int64_t no, const double* __restrict__ cams, const double* __restrict__ pts,
                          const int* __restrict__ oc, const int* __restrict__ op, double* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= no) return;
  const double* b = cams + 9 * (size_t)oc[i];
  Cam<double> c;
  so3_exp(b[0], b[1], b[2], c.R);
  c.t[0] = b[3];
  c.t[1] = b[4];
  c.t[2] = b[5];
  c.f = b[6];
  c.k1 = b[7];
  c.k2 = b[8];
  const double* X = pts + 3 * (size_t)op[i];
  double u0, u1;
  snavely_residual<double>(c, X[0], X[1], X[2], 0.0, 0.0, u0, u1);
  out[2 * i] = u0;
  out[2 * i + 1] = u1;
}

static inline unsigned blocks_for(int64_t n, int threads) {
  return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads);
}

// Point-major pixels in float32 (float32-mixed form only).
static void cast_pixels(caspar_ba* h) {
  if (h->prec == CASPAR_FP64 || h->no == 0) return;
  k_px_cast<<<blocks_for(h->no, 256), 256, 0, h->stream>>>(h->no, reinterpret_cast<const double2*>(h->px),
                                                           static_cast<float2*>(h->px_s));
  CBA_LAUNCHED();
}

void sync(caspar_ba* h) { CBA_HIP(hipStreamSynchronize(h->stream)); }

// One wave stores the scalars into mapped host memory (one 32-bit word per
// lane), waits for its stores to reach system scope, then lane 0 publishes
// seq.  A host that sees seq therefore sees the whole struct, and since the
// stream runs in order, every kernel enqueued before this one has finished.
__global__ __launch_bounds__(64) void k_scalars_out(const DevScalars* __restrict__ s, DevScalars* host,
                                                    unsigned* flag, unsigned seq) {
  constexpr int kWords = (int)(sizeof(DevScalars) / 4);
  static_assert(kWords <= 64, "one word per lane");
  const int t = threadIdx.x;
  if (t < kWords) reinterpret_cast<volatile unsigned*>(host)[t] = reinterpret_cast<const unsigned*>(s)[t];
  __threadfence_system();
  if (t == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The mapped read-back costs one small kernel and a poll of host memory; a
// copy-engine transfer plus a stream synchronisation costs tens of
// microseconds more, several times per Levenberg-Marquardt iteration.  A
// handle on the static workspace has no pinned memory and copies into its
// own struct instead.
DevScalars read_scalars(caspar_ba* h) {
  if (!h->scal_flag) {
    CBA_HIP(hipMemcpyAsync(h->scal_host, h->scal, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream));
    sync(h);
    return *h->scal_host;
  }
  const unsigned seq = ++h->scal_seq;
  k_scalars_out<<<1, 64, 0, h->stream>>>(
      h->scal, reinterpret_cast<DevScalars*>(h->scal_mapped_dev),
      reinterpret_cast<unsigned*>(h->scal_mapped_dev + sizeof(DevScalars) + 64), seq);
  CBA_LAUNCHED();
  for (unsigned spin = 1;; ++spin) {
    if (__atomic_load_n(h->scal_flag, __ATOMIC_ACQUIRE) == seq) break;
    if ((spin & 4095u) == 0) {
      // a failed kernel never publishes: ask the stream now and then
      const hipError_t e = hipStreamQuery(h->stream);
      if (e == hipSuccess) {
        if (__atomic_load_n(h->scal_flag, __ATOMIC_ACQUIRE) == seq) break;
        fail(CASPAR_EHIP, "scalar read-back: the stream finished without publishing");
      }
      if (e != hipErrorNotReady) CBA_HIP(e);
    }
  }
  DevScalars out;
  std::memcpy(&out, (const void*)h->scal_host, sizeof(DevScalars));
  return out;
}

void upload_cameras_bal(caspar_ba* h, const double* bal, double* cam) {
  if (h->nc == 0) return;
  k_cams_from_bal<<<blocks_for(h->nc, 256), 256, 0, h->stream>>>(h->nc, bal, h->cam_c2i, cam);
  CBA_LAUNCHED();
}

void upload_points(caspar_ba* h, const double* pts, double* X) {
  if (h->np == 0) return;
  k_points_in<<<blocks_for(h->np, 256), 256, 0, h->stream>>>(h->np, pts, h->pt_c2i, X);
  CBA_LAUNCHED();
}

template <typename V>
static void h2d(caspar_ba* h, V* dst, const std::vector<V>& src) {
  if (src.empty()) return;
  CBA_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice, h->stream));
  sync(h);  // the host vector may change or die right after
}

template <typename V>
static std::vector<V> d2h(caspar_ba* h, const V* src, size_t n) {
  std::vector<V> out(n);
  if (n) {
    CBA_HIP(hipMemcpyAsync(out.data(), src, n * sizeof(V), hipMemcpyDeviceToHost, h->stream));
    sync(h);
  }
  return out;
}

// Per-observation values (the meta words at create, the IRLS weights after
// each robust linearisation) in the point-per-lane product's step order.
// Lane l of lane tile t holds unit 64 t + l (k observations) and at step i
// visits its observation (i + l mod k) mod k; past its k observations, and on
// lanes past the last unit (whose k is 0; they read the last unit's), its
// first one.  The value goes to (lane_base[t] + i) * 64 + l, so that the 64
// lanes of a step read 64 consecutive values.  The cold-row numbering built at
// create walks each tile's cameras in this same order, so the two change
// together.
template <typename T>
__global__ void k_lane_order(int n_tiles, int n_units, const int* __restrict__ unit_obs,
                             const int* __restrict__ lane_base, const T* __restrict__ meta,
                             T* __restrict__ out) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)n_tiles * kWave) return;
  const int t = (int)(gid / kWave), lane = (int)(gid % kWave);
  const int u = t * kWave + lane;
  const bool valid = u < n_units;
  const int uc = valid ? u : n_units - 1;
  const int ob = unit_obs[uc];
  const int k = valid ? unit_obs[uc + 1] - ob : 0;
  const int rot = k > 0 ? lane % k : 0;
  const int b = lane_base[t], trip = lane_base[t + 1] - b;
  for (int i = 0; i < trip; ++i) {
    int j = i + rot;
    if (j >= k) j -= k;
    out[((size_t)b + i) * kWave + lane] = meta[i < k ? ob + j : ob];
  }
}

void launch_lane_weights(caspar_ba* h) {
  if (!h->rj || h->n_lane_tiles == 0) return;
  const unsigned g = blocks_for((int64_t)h->n_lane_tiles * kWave, 256);
  if (h->prec == CASPAR_FP64)
    k_lane_order<double><<<g, 256, 0, h->stream>>>(h->n_lane_tiles, h->n_units, h->unit_obs, h->lane_base,
                                                   (const double*)h->wts, (double*)h->lane_wts);
  else
    k_lane_order<float><<<g, 256, 0, h->stream>>>(h->n_lane_tiles, h->n_units, h->unit_obs, h->lane_base,
                                                  (const float*)h->wts, (float*)h->lane_wts);
  CBA_LAUNCHED();
}

static void build_layout(caspar_ba* h, const double* cams, const double* pts, const int* oc,
                         const int* op, const double* px_caller, char* ws, const Plan& plan) {
  const int nc = h->nc, np = h->np, no = h->no;
  hipStream_t st = h->stream;

  // Create-time scratch inside the J region.
  char* scratch = (char*)h->J;
  size_t so = 0;
  auto carve = [&](size_t bytes) {
    char* p = scratch + so;
    so += align_up(bytes);
    return (void*)p;
  };
  uint64_t* keys_a = (uint64_t*)carve(8 * (size_t)no);
  uint64_t* keys_b = (uint64_t*)carve(8 * (size_t)no);
  int* vals_a = (int*)carve(4 * (size_t)no);
  int* vals_b = (int*)carve(4 * (size_t)no);
  const size_t cub_bytes = sort_temp_bytes(no);
  void* cub_tmp = carve(cub_bytes);
  int* pt_cnt = (int*)carve(4 * (size_t)np);
  int* pt_key = (int*)carve(4 * (size_t)np);
  int* cam_cnt = (int*)carve(4 * (size_t)nc);
  if (so > plan.J.bytes) fail(CASPAR_ENOMEM, "internal: create scratch exceeds plan");
  int* cm_obs = h->cm_obs;

  // Validation.
  CBA_HIP(hipMemsetAsync(h->scal, 0, sizeof(DevScalars), st));
  {
    const int64_t n = std::max<int64_t>({(int64_t)no, (int64_t)nc * 9, (int64_t)np * 3, 1});
    k_validate<<<blocks_for(n, 256), 256, 0, st>>>(nc, np, no, cams, pts, oc, op, px_caller, h->scal);
    CBA_LAUNCHED();
    const DevScalars s = read_scalars(h);
    if (s.err & 1) fail(CASPAR_EINVAL, "observation camera or point index out of range");
    if (s.err & 2) fail(CASPAR_EINVAL, "non-finite observed pixel");
    if (s.err & 4) fail(CASPAR_EINVAL, "non-finite camera parameter");
    if (s.err & 8) fail(CASPAR_EINVAL, "non-finite point coordinate");
  }

  // Camera relabelling by observation count.
  if (nc) CBA_HIP(hipMemsetAsync(cam_cnt, 0, 4 * (size_t)nc, st));
  if (np) CBA_HIP(hipMemsetAsync(pt_cnt, 0, 4 * (size_t)np, st));
  if (no) {
    const bool lds_hist = nc <= kCountLdsCams;
    if (lds_hist) {
      const size_t lds = (size_t)nc * sizeof(int);
      if (lds > 65536)
        CBA_HIP(hipFuncSetAttribute((const void*)k_count_cams, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      k_count_cams<<<std::min<unsigned>(blocks_for(no, 1024), kNumCUs), 1024, lds, st>>>(no, oc, nc, cam_cnt);
      CBA_LAUNCHED();
    }
    k_count<<<blocks_for(no, 256), 256, 0, st>>>(no, oc, op, lds_hist ? nullptr : cam_cnt, pt_cnt);
    CBA_LAUNCHED();
  }
  std::vector<int> ccnt = d2h(h, cam_cnt, nc);
  std::vector<int> cam_i2c(nc), cam_c2i(nc);
  std::iota(cam_i2c.begin(), cam_i2c.end(), 0);
  std::stable_sort(cam_i2c.begin(), cam_i2c.end(), [&](int a, int b) { return ccnt[a] > ccnt[b]; });
  for (int i = 0; i < nc; ++i) cam_c2i[cam_i2c[i]] = i;
  h2d(h, h->cam_c2i, cam_c2i);
  h2d(h, h->cam_i2c, cam_i2c);

  // Point order: by least-observed camera (largest internal id), then id.
  if (np) CBA_HIP(hipMemsetAsync(pt_key, 0xff, 4 * (size_t)np, st));  // -1
  if (no) {
    k_point_key<<<blocks_for(no, 256), 256, 0, st>>>(no, oc, op, h->cam_c2i, pt_key);
    CBA_LAUNCHED();
  }
  std::vector<int> pkey = d2h(h, pt_key, np);
  std::vector<int> pcnt = d2h(h, pt_cnt, np);
  std::vector<int> pt_i2c(np), pt_c2i(np);
  {
    std::vector<int> bucket(nc + 2, 0);
    for (int p = 0; p < np; ++p) bucket[pkey[p] + 2]++;
    for (int i = 1; i < nc + 2; ++i) bucket[i] += bucket[i - 1];
    for (int p = 0; p < np; ++p) pt_i2c[bucket[pkey[p] + 1]++] = p;
    for (int i = 0; i < np; ++i) pt_c2i[pt_i2c[i]] = i;
  }
  h2d(h, h->pt_c2i, pt_c2i);
  h2d(h, h->pt_i2c, pt_i2c);
  int n_orphan = 0;
  while (n_orphan < np && pcnt[pt_i2c[n_orphan]] == 0) ++n_orphan;
  h->n_orphan_pts = n_orphan;

  // Wave tiles (greedy packing of whole points) and split points.
  std::vector<Tile> tiles;
  std::vector<SplitPoint> splits;
  {
    int64_t off = 0;
    Tile cur{};
    int cur_n = 0, cur_pts = 0, cur_max = 0;
    auto steps = [](int m) { return m <= 1 ? 0 : ceil_log2(m); };
    auto flush = [&]() {
      if (cur_n == 0) return;
      cur.info = cur_n | (cur_pts << 7) | (steps(cur_max) << 14);
      cur.split_row = -1;
      tiles.push_back(cur);
      cur_n = cur_pts = cur_max = 0;
    };
    int split_row = 0;
    for (int i = n_orphan; i < np; ++i) {
      const int k = pcnt[pt_i2c[i]];
      if (k > kTileMax) {
        flush();
        SplitPoint sp{i, split_row, 0, 0};
        for (int s0 = 0; s0 < k; s0 += kTileMax) {
          Tile t{};
          const int n = std::min(kTileMax, k - s0);
          t.obs_begin = (int)(off + s0);
          t.pt_begin = i;
          t.split_row = split_row++;
          t.info = n | (1 << 7) | (steps(n) << 14) | (1 << 17) | ((s0 == 0 ? 1 : 0) << 18);
          tiles.push_back(t);
          sp.nrows++;
        }
        splits.push_back(sp);
      } else {
        if (cur_n + k > kTileMax) flush();
        if (cur_n == 0) {
          cur = Tile{};
          cur.obs_begin = (int)off;
          cur.pt_begin = i;
        }
        cur_n += k;
        cur_pts += 1;
        cur_max = std::max(cur_max, k);
      }
      off += k;
    }
    flush();
    if (off != no) fail(CASPAR_EINVAL, "internal: observation count mismatch");
  }
  if (tiles.size() > plan.max_tiles || splits.size() > plan.max_split_pts)
    fail(CASPAR_ENOMEM, "internal: tile table exceeds plan");
  h->n_tiles = (int)tiles.size();
  h->n_split_pts = (int)splits.size();
  h->n_split_tiles = splits.empty() ? 0 : splits.back().row_begin + splits.back().nrows;
  if ((size_t)h->n_split_tiles > plan.max_split_tiles) fail(CASPAR_ENOMEM, "internal: split rows");
  h2d(h, h->split_pts, splits);

  // Lane units of the point-per-lane kernels (the linearisation, and the
  // product with recomputed blocks): whole points of at most kLaneObsMax
  // observations, pieces of the others; 64 units per wave tile, whose trip
  // count is its largest unit.
  std::vector<int> unit_obs, unit_pt, unit_row;
  std::vector<int2> lane_tiles;
  if (no) {
    std::vector<SplitPoint> lsplits;
    int64_t off = 0;
    int row = 0;
    for (int i = n_orphan; i < np; ++i) {
      const int k = pcnt[pt_i2c[i]];
      if (k <= kLaneObsMax) {
        unit_obs.push_back((int)off);
        unit_pt.push_back(i);
        unit_row.push_back(-1);
      } else {
        SplitPoint sp{i, row, 0, 0};
        for (int s0 = 0; s0 < k; s0 += kLaneObsMax) {
          unit_obs.push_back((int)(off + s0));
          unit_pt.push_back((int)((unsigned)i | (1u << 31) | ((s0 == 0 ? 1u : 0u) << 30)));
          unit_row.push_back(row++);
          sp.nrows++;
        }
        lsplits.push_back(sp);
      }
      off += k;
    }
    unit_obs.push_back((int)off);
    h->n_units = (int)unit_pt.size();
    h->n_lane_tiles = (h->n_units + kWave - 1) / kWave;
    h->n_lane_split_pts = (int)lsplits.size();
    if ((size_t)h->n_units > plan.max_units || (size_t)h->n_lane_tiles > plan.max_lane_tiles ||
        lsplits.size() > plan.max_lane_split_pts || (size_t)row > plan.max_pieces)
      fail(CASPAR_ENOMEM, "internal: lane units exceed plan");
    // trip counts of at least two: the product looks two iterations ahead,
    // into this tile or the next
    lane_tiles.assign(h->n_lane_tiles, make_int2(2, 0));
    for (int u = 0; u < h->n_units; ++u) {
      int2& lt = lane_tiles[u / kWave];
      lt.x = std::max(lt.x, unit_obs[u + 1] - unit_obs[u]);
    }
    h2d(h, h->unit_obs, unit_obs);
    h2d(h, h->unit_pt, unit_pt);
    h2d(h, h->unit_row, unit_row);
    h2d(h, h->lane_split_pts, lsplits);
  }

  // Point-major sort of the observations.
  const int pt_bits = std::max(1, ceil_log2((long long)np + 1));
  const int cam_bits = std::max(1, ceil_log2((long long)nc + 1));
  if (no) {
    k_make_keys<<<blocks_for(no, 256), 256, 0, st>>>(no, oc, op, h->cam_c2i, h->pt_c2i, keys_a, vals_a);
    CBA_LAUNCHED();
    size_t tb = cub_bytes;
    CBA_HIP(hipcub::DeviceRadixSort::SortPairs(cub_tmp, tb, keys_a, keys_b, vals_a, h->obs_s2c, no, 0,
                                               kCamBits + pt_bits, st));
    h2d(h, h->tiles, tiles);
    k_fill_obs<<<blocks_for((int64_t)h->n_tiles * kWave, 256), 256, 0, st>>>(
        h->n_tiles, h->tiles, keys_b, h->obs_s2c, px_caller, h->meta, h->px, (uint32_t*)keys_a,
        vals_a);
    CBA_LAUNCHED();
    // Camera-major order (stable: inside a camera, point order).
    tb = cub_bytes;
    CBA_HIP(hipcub::DeviceRadixSort::SortPairs(cub_tmp, tb, (const uint32_t*)keys_a, (uint32_t*)vals_b,
                                               vals_a, cm_obs, no, 0, cam_bits, st));
    if (h->prec == CASPAR_FP64)
      k_fill_cm<double><<<blocks_for(no, 256), 256, 0, st>>>(no, cm_obs, keys_b, h->px, h->cm_pt, h->cm_px);
    else
      k_fill_cm<float><<<blocks_for(no, 256), 256, 0, st>>>(no, cm_obs, keys_b, h->px, h->cm_pt,
                                                            static_cast<float*>(h->cm_px_s));
    CBA_LAUNCHED();
    cast_pixels(h);
  }

  // Camera offsets (internal order) and linearisation chunks.  A camera's
  // entries are cut into chunks of kCamChunk, one workgroup each, while more
  // than kCamSmallChunk remain; a rest of at most kCamSmallChunk entries
  // (the whole camera, for most cameras of a heavy-tailed scene) is a small
  // chunk that one wave sums, four to a workgroup.  The table holds the
  // workgroup chunks first; each chunk's output row keeps the rows of a
  // camera consecutive.  A camera's entries are in point order, and the
  // points of a much-observed camera spread over the whole point order, so
  // the workgroup chunks are launched in the order of where they sit inside
  // their camera (the middle entry's fraction of the camera's entries): the
  // chunks in flight together gather from one region of the points, which
  // then stays in the L2 caches, instead of each camera's chunks sweeping
  // all points in turn.
  std::vector<int> cam_off(nc + 1, 0), chunk_off(nc + 1, 0);
  std::vector<Chunk> chunks, small;
  std::vector<std::pair<double, int>> order;  // (position inside the camera, chunk)
  int row = 0;
  for (int i = 0; i < nc; ++i) {
    const int n = ccnt[cam_i2c[i]];
    cam_off[i + 1] = cam_off[i] + n;
    int b = 0;
    for (; n - b > kCamSmallChunk; b += kCamChunk) {
      const int e = std::min(n, b + kCamChunk);
      order.emplace_back(0.5 * (b + e) / n, (int)chunks.size());
      chunks.push_back(Chunk{i, cam_off[i] + b, cam_off[i] + e, row++});
    }
    if (b < n) small.push_back(Chunk{i, cam_off[i] + b, cam_off[i] + n, row++});
    chunk_off[i + 1] = row;
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<double, int>& a, const std::pair<double, int>& b) { return a.first < b.first; });
  {
    std::vector<Chunk> sorted;
    sorted.reserve(chunks.size());
    for (const auto& o : order) sorted.push_back(chunks[o.second]);
    chunks.swap(sorted);
  }
  h->n_big_chunks = (int)chunks.size();
  chunks.insert(chunks.end(), small.begin(), small.end());
  if (chunks.size() > plan.max_chunks) fail(CASPAR_ENOMEM, "internal: chunk table exceeds plan");
  h->n_chunks = (int)chunks.size();
  h2d(h, h->cam_off, cam_off);
  h2d(h, h->chunk_off, chunk_off);
  h2d(h, h->chunks, chunks);

  // Fused-product grid: workgroup g takes tiles [n_tiles g / G, n_tiles (g + 1) / G).
  const int waves = matvec_waves(h->prec, h->rj);
  const bool lane_mode = h->rj;  // the product runs point-per-lane over the lane tiles
  const int n_ptiles = lane_mode ? h->n_lane_tiles : h->n_tiles;
  h->L = nc > h->K ? std::min(kColdWin, nc - h->K) : 0;
  // a point-per-lane product that would give fewer workgroups than CUs runs
  // four-wave workgroups instead: more of them, each with fewer tiles
  h->mv_small = lane_mode && (n_ptiles + waves - 1) / waves < kNumCUs;
  const int wg_waves = h->mv_small ? matvec_small_waves() : waves;
  h->G = std::max(1, std::min(groups_per_cu(h->K, h->L) * kNumCUs, (n_ptiles + wg_waves - 1) / wg_waves));

  // Cold cameras (internal id >= K).  Points are ordered by their least
  // observed camera, so the cold observations of one workgroup's tiles
  // concentrate on a narrow band of camera ids: each workgroup gets the
  // window of L consecutive cold cameras holding most of its cold
  // observations and sums them in LDS (rows local_base + g L + slot).  Every
  // other cold observation writes a row of its own: per tile, rows
  // cold_begin, cold_begin + 1, ... in lane order.  Per camera: its rows.
  h->n_cold = (nc > h->K) ? cam_off[nc] - cam_off[h->K] : 0;
  h->n_cold_rows = 0;
  h->cold_local_base = 0;
  if (h->n_cold > 0) {
    std::vector<uint32_t> meta_h = d2h(h, h->meta, (size_t)no);
    const int K = h->K, L = h->L, G = h->G;
    auto cam_at = [&](int64_t o) { return (int)(meta_h[o] & ((1u << kCamBits) - 1)); };
    // the cameras of product tile t in the order the kernel visits them: lane
    // order (observation per lane), or iteration-major, lane-minor with each
    // unit's observations rotated by lane mod k (point per lane)
    auto tile_cams = [&](int t, auto&& f) {
      if (!lane_mode) {
        for (int lane = 0; lane < tile_nobs(tiles[t].info); ++lane) f(cam_at(tiles[t].obs_begin + lane));
        return;
      }
      const int u0 = t * kWave, u1 = std::min(h->n_units, u0 + kWave);
      for (int it = 0; it < lane_tiles[t].x; ++it)
        for (int u = u0; u < u1; ++u) {
          const int ob = unit_obs[u], k = unit_obs[u + 1] - ob;
          if (it >= k) continue;
          int j = it + (u - u0) % k;
          if (j >= k) j -= k;
          f(cam_at((int64_t)ob + j));
        }
    };
    auto set_cold_begin = [&](int t, int v) {
      if (lane_mode)
        lane_tiles[t].y = v;
      else
        tiles[t].cold_begin = v;
    };
    std::vector<int> lo(G, K);
    std::vector<std::vector<int>> rows_of(nc - K);
    std::vector<int> ids;
    int run = 0, n_cold_seen = 0;
    for (int g = 0; g < G; ++g) {
      const int t0 = (int)((int64_t)n_ptiles * g / G), t1 = (int)((int64_t)n_ptiles * (g + 1) / G);
      ids.clear();
      for (int t = t0; t < t1; ++t)
        tile_cams(t, [&](int c) {
          if (c >= K) ids.push_back(c);
        });
      std::sort(ids.begin(), ids.end());
      // window [lo, lo + L) holding the most of this workgroup's cold observations
      int best = 0;
      for (size_t i = 0, j = 0; i < ids.size(); ++i) {
        while (j < ids.size() && ids[j] < ids[i] + L) ++j;
        if ((int)(j - i) > best) {
          best = (int)(j - i);
          lo[g] = std::min(ids[i], nc - L);
        }
      }
      for (int t = t0; t < t1; ++t) {
        set_cold_begin(t, run);
        tile_cams(t, [&](int c) {
          if (c < K) return;
          ++n_cold_seen;
          if (c < lo[g] || c >= lo[g] + L) rows_of[c - K].push_back(run++);
        });
      }
    }
    if (n_cold_seen != h->n_cold) fail(CASPAR_EINVAL, "internal: cold count mismatch");
    if ((size_t)run > plan.max_cold || G > kMaxGroups) fail(CASPAR_ENOMEM, "internal: cold rows exceed plan");
    // window rows, listed for the cameras that have observations in them
    h->cold_local_base = run;
    for (int g = 0; g < G; ++g) {
      std::vector<char> used(L, 0);
      const int t0 = (int)((int64_t)n_ptiles * g / G), t1 = (int)((int64_t)n_ptiles * (g + 1) / G);
      for (int t = t0; t < t1; ++t)
        tile_cams(t, [&](int c) {
          if (c >= K && c >= lo[g] && c < lo[g] + L) used[c - lo[g]] = 1;
        });
      for (int sl = 0; sl < L; ++sl)
        if (used[sl]) rows_of[lo[g] + sl - K].push_back(run + g * L + sl);
    }
    h->n_cold_rows = run + G * L;
    const size_t scat_bytes = (size_t)run * (h->prec == CASPAR_FP64 ? ColdRow<double>::n * 8 : ColdRow<float>::n * 4);
    if (scat_bytes >= ((size_t)1 << 31))
      fail(CASPAR_EINVAL, "too many observations of rarely observed cameras: the product's row buffer exceeds 2 GiB");
    h->win_rows = reinterpret_cast<double*>(static_cast<char*>(h->cold_rows) + align_up(scat_bytes));
    std::vector<int> coff(nc - K + 1, 0), clist;
    for (int c = K; c < nc; ++c) {
      coff[c - K + 1] = coff[c - K] + (int)rows_of[c - K].size();
      clist.insert(clist.end(), rows_of[c - K].begin(), rows_of[c - K].end());
    }
    h2d(h, h->cold_lo, lo);
    h2d(h, h->cold_off, coff);
    h2d(h, h->cold_list, clist);
  }
  if (no) h2d(h, h->tiles, tiles);
  h2d(h, h->lane_tiles, lane_tiles);

  // Recomputed blocks: the meta words of the point-per-lane kernels in their
  // step order.
  if (no && h->rj) {
    std::vector<int> lbase(h->n_lane_tiles + 1, 0);
    for (int t = 0; t < h->n_lane_tiles; ++t) lbase[t + 1] = lbase[t] + lane_tiles[t].x;
    if ((size_t)lbase.back() > plan.max_lane_tiles * kLaneObsMax) fail(CASPAR_ENOMEM, "internal: lane steps exceed plan");
    h2d(h, h->lane_base, lbase);
    k_lane_order<uint32_t><<<blocks_for((int64_t)h->n_lane_tiles * kWave, 256), 256, 0, st>>>(
        h->n_lane_tiles, h->n_units, h->unit_obs, h->lane_base, h->meta, h->lane_meta);
    CBA_LAUNCHED();
  }

  // Parameters.
  upload_cameras_bal(h, cams, h->cam);
  upload_points(h, pts, h->X);
  sync(h);
}

}  // namespace cba

// Static workspace for callers that cannot allocate (caspar_ba_create_static):
// one file-scope device array, each GPU holding its own copy for the life of
// the process.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.  One
// handle at a time may hold a device's array; the claim is released when that
// handle is destroyed.
static __device__ __align__(256) unsigned char scratch[cba::kStaticWorkspaceBytes];

namespace {
std::mutex g_static_mu;
std::vector<void*> g_static_ptr;   // per device: scratch's device address (nullptr: not looked up)
std::vector<char> g_static_held;   // per device: held by a live handle
}  // namespace

namespace cba {
void* static_workspace_claim(int dev) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  if ((size_t)dev >= g_static_ptr.size()) {
    g_static_ptr.resize((size_t)dev + 1, nullptr);
    g_static_held.resize((size_t)dev + 1, 0);
  }
  if (g_static_held[dev])
    fail(CASPAR_EINVAL, "the static workspace of this GPU is held by another handle (destroy it first)");
  if (g_static_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      fail(CASPAR_EHIP, std::string("hipGetSymbolAddress of the static workspace failed: ") + hipGetErrorString(e));
    g_static_ptr[dev] = ptr;
  }
  g_static_held[dev] = 1;
  return g_static_ptr[dev];
}

void static_workspace_release(int dev) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (dev >= 0 && (size_t)dev < g_static_held.size()) g_static_held[dev] = 0;
}
}  // namespace cba

namespace cba {

// create() on a given workspace.  static_dev >= 0: the workspace is that
// device's static array (no host staging buffer is allocated either; scalar
// read-backs land in the handle itself).
static int create_impl(caspar_ba** out, int32_t n_cams, int32_t n_points, int64_t n_obs, const double* cams,
                       const double* points, const int32_t* obs_cam, const int32_t* obs_pt, const double* obs_px,
                       int mode, void* workspace, size_t workspace_bytes, void* hip_stream, int static_dev) {
  caspar_ba* h = nullptr;
  try {
    CBA_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    Plan plan;
    CBA_REQUIRE(make_plan(n_cams, n_points, n_obs, mode, plan),
                "bad sizes or mode (n_obs < 2^31, n_cams < 2^25, observations need cameras and points)");
    if (static_dev >= 0) {
      if (plan.total > kStaticWorkspaceBytes)
        fail(CASPAR_ENOMEM, "problem needs " + std::to_string(plan.total) +
                                " bytes of workspace; the static workspace holds " +
                                std::to_string(kStaticWorkspaceBytes) + " (use caspar_ba_create)");
      workspace = static_workspace_claim(static_dev);
      workspace_bytes = kStaticWorkspaceBytes;
    }
    if (workspace_bytes < plan.total)
      fail(CASPAR_ENOMEM, "workspace too small: need " + std::to_string(plan.total) + " bytes");
    CBA_REQUIRE(workspace != nullptr && ((uintptr_t)workspace & 255) == 0,
                "workspace must be non-NULL and 256-byte aligned");
    CBA_REQUIRE(n_obs == 0 || (obs_cam && obs_pt && obs_px), "observation arrays are NULL");
    CBA_REQUIRE(n_cams == 0 || cams, "cams is NULL");
    CBA_REQUIRE(n_points == 0 || points, "points is NULL");
    h = new caspar_ba();
    h->static_dev = static_dev;
    static_dev = -1;  // released by the handle from here on
    h->nc = n_cams;
    h->np = n_points;
    h->no = (int)n_obs;
    h->prec = mode & 1;
    h->rj = (mode & CASPAR_RECOMPUTE_JACOBIAN) != 0;
    h->N = 9 * n_cams + 3 * n_points;
    h->stream = (hipStream_t)hip_stream;
    h->no_pad = (int)align_up((size_t)n_obs, kJBlock);
    h->K = plan.K;
    CBA_HIP(hipGetDevice(&h->device));
    char* ws = (char*)workspace;
    h->scal = (DevScalars*)(ws + plan.scal.off);
    if (h->static_dev >= 0) {
      h->scal_host = &h->scal_local;
    } else {
      // the struct, then the flag on a line of its own
      char* pinned = nullptr;
      CBA_HIP(hipHostMalloc((void**)&pinned, sizeof(DevScalars) + 128, hipHostMallocMapped | hipHostMallocCoherent));
      h->scal_host = reinterpret_cast<DevScalars*>(pinned);
      h->scal_flag = reinterpret_cast<unsigned*>(pinned + sizeof(DevScalars) + 64);
      *h->scal_flag = 0;
      CBA_HIP(hipHostGetDevicePointer((void**)&h->scal_mapped_dev, pinned, 0));
    }
    h->partials = (double*)(ws + plan.partials.off);
    h->gauge_rows = (double*)(ws + plan.gauge_rows.off);
    h->cam = (double*)(ws + plan.cam.off);
    h->cam_trial = (double*)(ws + plan.cam_trial.off);
    h->cam_s = ws + plan.cam_s.off;
    h->cam_trial_s = ws + plan.cam_trial_s.off;
    h->pts_s = ws + plan.pts_s.off;
    h->wts = ws + plan.wts.off;
    h->X = (double*)(ws + plan.X.off);
    h->X_trial = (double*)(ws + plan.X_trial.off);
    h->cam_c2i = (int*)(ws + plan.cam_c2i.off);
    h->cam_i2c = (int*)(ws + plan.cam_i2c.off);
    h->pt_c2i = (int*)(ws + plan.pt_c2i.off);
    h->pt_i2c = (int*)(ws + plan.pt_i2c.off);
    h->obs_s2c = (int*)(ws + plan.obs_s2c.off);
    h->meta = (uint32_t*)(ws + plan.meta.off);
    h->px = (double*)(ws + plan.px.off);
    h->J = ws + plan.J.off;
    h->tiles = (Tile*)(ws + plan.tiles.off);
    h->cold_lo = (int*)(ws + plan.cold_lo.off);
    h->p_cam = ws + plan.p_cam.off;
    h->cm_obs = (int*)(ws + plan.cm_obs.off);
    h->cm_pt = (int*)(ws + plan.cm_pt.off);
    h->cm_px = (double*)(ws + plan.cm_px.off);
    h->px_s = ws + plan.px_s.off;
    h->cm_px_s = ws + plan.cm_px_s.off;
    h->cam_off = (int*)(ws + plan.cam_off.off);
    h->chunks = (Chunk*)(ws + plan.chunks.off);
    h->chunk_off = (int*)(ws + plan.chunk_off.off);
    h->chunk_rows = (double*)(ws + plan.chunk_rows.off);
    h->cold_list = (int*)(ws + plan.cold_list.off);
    h->cold_off = (int*)(ws + plan.cold_off.off);
    h->cold_rows = ws + plan.cold_rows.off;
    h->split_pts = (SplitPoint*)(ws + plan.split_pts.off);
    h->split_rows = (double*)(ws + plan.split_rows.off);
    h->unit_obs = (int*)(ws + plan.unit_obs.off);
    h->unit_pt = (int*)(ws + plan.unit_pt.off);
    h->unit_row = (int*)(ws + plan.unit_row.off);
    h->lane_tiles = (int2*)(ws + plan.lane_tiles.off);
    h->lane_split_pts = (SplitPoint*)(ws + plan.lane_split_pts.off);
    h->lane_split_rows = (double*)(ws + plan.lane_split_rows.off);
    h->lane_base = (int*)(ws + plan.lane_base.off);
    h->lane_meta = (uint32_t*)(ws + plan.lane_meta.off);
    h->lane_wts = ws + plan.lane_wts.off;
    h->hot_rows = ws + plan.hot_rows.off;
    h->Hcc = (double*)(ws + plan.Hcc.off);
    h->Hpp = (double*)(ws + plan.Hpp.off);
    h->Mc = ws + plan.Mc.off;
    h->Mp = ws + plan.Mp.off;
    void** vp[8] = {&h->vec.g, &h->vec.D, &h->vec.x, &h->vec.r, &h->vec.z, &h->vec.p, &h->vec.w, &h->vec.v};
    for (int i = 0; i < 8; ++i) *vp[i] = ws + plan.vecs.off + i * plan.vec_bytes;
    build_layout(h, cams, points, obs_cam, obs_pt, obs_px, ws, plan);
    *out = h;
  } catch (const Error& e) {
    delete h;
    if (static_dev >= 0) static_workspace_release(static_dev);
    set_last_error(e.msg);
    return e.status;
  } catch (const std::exception& e) {
    delete h;
    if (static_dev >= 0) static_workspace_release(static_dev);
    set_last_error(e.what());
    return CASPAR_EHIP;
  }
  set_last_error("");
  return CASPAR_OK;
}

}  // namespace cba

caspar_ba::~caspar_ba() {
  if (scal_host && static_dev < 0) (void)hipHostFree(scal_host);
  if (static_dev >= 0) cba::static_workspace_release(static_dev);
  for (hipEvent_t e : ev_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : ev_stop) (void)hipEventDestroy(e);
}

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

const char* caspar_last_error(void) { return g_last_error.c_str(); }

void caspar_default_solve_opts(caspar_solve_opts* o) {
  if (!o) return;
  o->lambda0 = 1e-2;
  o->pcg_tol = 1e-3;
  o->max_lm_iters = 20;
  o->max_pcg_iters = 500;
  o->lambda_min = 1e-12;
  o->lambda_max = 1e16;
  o->grad_tol = 1e-12;
  o->min_cost = 1e-30;
  o->pcg_check_every = 4;
  o->flags = 0;
  o->pred_tol = 0.0;
}

size_t caspar_ba_workspace_bytes(int32_t n_cams, int32_t n_points, int64_t n_obs, int mode) {
  Plan p;
  if (!make_plan(n_cams, n_points, n_obs, mode, p)) return 0;
  return p.total;
}

int caspar_ba_create(caspar_ba** out, int32_t n_cams, int32_t n_points, int64_t n_obs,
                     const double* cams, const double* points, const int32_t* obs_cam,
                     const int32_t* obs_pt, const double* obs_px, int mode, void* workspace,
                     size_t workspace_bytes, void* hip_stream) {
  return create_impl(out, n_cams, n_points, n_obs, cams, points, obs_cam, obs_pt, obs_px, mode, workspace,
                     workspace_bytes, hip_stream, -1);
}

int caspar_ba_create_static(caspar_ba** out, int32_t n_cams, int32_t n_points, int64_t n_obs,
                            const double* cams, const double* points, const int32_t* obs_cam,
                            const int32_t* obs_pt, const double* obs_px, int mode, void* hip_stream) {
  int dev = -1;
  if (out) *out = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    set_last_error("hipGetDevice failed");
    return CASPAR_EHIP;
  }
  return create_impl(out, n_cams, n_points, n_obs, cams, points, obs_cam, obs_pt, obs_px, mode, nullptr, 0,
                     hip_stream, dev);
}

void caspar_ba_destroy(caspar_ba* h) { delete h; }

int caspar_ba_get_params(caspar_ba* h, double* cams, double* points) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  if (cams && h->nc) {
    k_cams_to_bal<<<blocks_for(h->nc, 256), 256, 0, h->stream>>>(h->nc, h->cam, h->cam_c2i, cams);
    CBA_LAUNCHED();
  }
  if (points && h->np) {
    k_points_out<<<blocks_for(h->np, 256), 256, 0, h->stream>>>(h->np, h->X, h->pt_c2i, points);
    CBA_LAUNCHED();
  }
  sync(h);
  CBA_API_END
}

int caspar_ba_set_params(caspar_ba* h, const double* cams, const double* points) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  if (cams) upload_cameras_bal(h, cams, h->cam);
  if (points) upload_points(h, points, h->X);
  h->linearized = false;
  sync(h);
  CBA_API_END
}

int caspar_ba_set_loss(caspar_ba* h, int32_t kind, double scale) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  CBA_REQUIRE(kind == CASPAR_LOSS_TRIVIAL || kind == CASPAR_LOSS_HUBER || kind == CASPAR_LOSS_CAUCHY,
              "unknown loss kind");
  CBA_REQUIRE(std::isfinite(scale) && scale > 0.0, "loss scale must be finite and > 0");
  h->loss = kind;
  h->loss_c = scale;
  h->linearized = false;
  CBA_API_END
}

int caspar_ba_set_observations(caspar_ba* h, const double* obs_px) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  CBA_REQUIRE(h->no == 0 || obs_px != nullptr, "obs_px is NULL");
  if (h->no) {
    k_set_px<<<blocks_for(h->no, 256), 256, 0, h->stream>>>(h->no, h->obs_s2c, obs_px, h->px);
    CBA_LAUNCHED();
    if (h->prec == CASPAR_FP64)
      k_set_cm_px<double><<<blocks_for(h->no, 256), 256, 0, h->stream>>>(h->no, h->cm_obs, h->px, h->cm_px);
    else
      k_set_cm_px<float><<<blocks_for(h->no, 256), 256, 0, h->stream>>>(h->no, h->cm_obs, h->px,
                                                                        static_cast<float*>(h->cm_px_s));
    CBA_LAUNCHED();
    cast_pixels(h);
  }
  h->linearized = false;
  sync(h);
  CBA_API_END
}

int caspar_project(int32_t n_cams, int32_t n_points, int64_t n_obs, const double* cams,
                   const double* points, const int32_t* obs_cam, const int32_t* obs_pt,
                   double* px_out, void* hip_stream) {
  CBA_API_BEGIN
  CBA_REQUIRE(n_cams >= 0 && n_points >= 0 && n_obs >= 0, "negative size");
  if (n_obs == 0) return CASPAR_OK;
  CBA_REQUIRE(cams && points && obs_cam && obs_pt && px_out, "NULL argument");
  hipStream_t st = (hipStream_t)hip_stream;
  k_project<<<blocks_for(n_obs, 256), 256, 0, st>>>(n_obs, cams, points, obs_cam, obs_pt, px_out);
  CBA_LAUNCHED();
  CBA_HIP(hipStreamSynchronize(st));
  CBA_API_END
}

int caspar_ba_layout_info(caspar_ba* h, int32_t* hot_cams, int64_t* cold_obs, int64_t* n_tiles,
                          int32_t* matvec_groups) {
  CBA_API_BEGIN
  CBA_REQUIRE(h != nullptr, "handle is NULL");
  if (hot_cams) *hot_cams = h->K;
  if (cold_obs) *cold_obs = h->n_cold;
  if (n_tiles) *n_tiles = h->n_tiles;
  if (matvec_groups) *matvec_groups = h->G;
  CBA_API_END
}

}  // extern "C"
