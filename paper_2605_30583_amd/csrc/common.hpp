// Internal declarations shared by the HIP translation units of the
// bundle-adjustment library.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "caspar_ba.h"

namespace cba {

// ---------------------------------------------------------------------------
// Errors: every public entry point catches Error and maps it to a status.
// ---------------------------------------------------------------------------
struct Error {
  int status;
  std::string msg;
};

void set_last_error(const std::string& msg);
[[noreturn]] void fail(int status, const std::string& msg);

#define CBA_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      ::cba::fail(CASPAR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CBA_REQUIRE(cond, msg)                          \
  do {                                                  \
    if (!(cond)) ::cba::fail(CASPAR_EINVAL, (msg));     \
  } while (0)

// Checks the launch status of the kernel just enqueued.
#define CBA_LAUNCHED() CBA_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Sizes and layout constants.
// ---------------------------------------------------------------------------
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kTileMax = 64;         // observations per wave tile
constexpr int kCamStride = 16;       // doubles per camera row: R(9) t(3) f k1 k2 pad
constexpr int kCamChunk = 2048;      // camera-major entries per linearisation chunk
constexpr int kCamSmallChunk = 512;  // at most this many: one wave's chunk (4 per workgroup)
constexpr int kCamRowWidth = 54;     // g_c (9) + upper triangle of H_cc (45)
constexpr int kPtRowWidth = 9;       // g_p (3) + upper triangle of H_pp (6)
constexpr int kColdRow = 10;         // doubles per cold-camera window row (9 sums, padded to 80 bytes)
constexpr int kLdsBudget = 147456;   // bytes of LDS for hot-camera accumulators (144 KiB)
constexpr int kPrivCams = 12;        // most observed cameras with private LDS copies in the product
constexpr int kPrivCopies = 8;       // (copy = lane mod 8; with 2048 hot cameras and the window, the LDS
                                     // of a workgroup is then full to 128 bytes)
constexpr int kColdWin = 128;        // cold cameras per product workgroup accumulated in its LDS window
constexpr int kMaxHot = kLdsBudget / (9 * 8);  // 2048 cameras with float64 sums
constexpr int kMaxPartials = 4096;   // per-workgroup partial slots
constexpr int kPartialWidth = 4;     // doubles per partial slot
constexpr int kCamBits = 25;         // meta: camera id bits; local point in bits 25..30
constexpr int kNumCUs = 256;
constexpr int kMaxGroups = 2 * kNumCUs;  // workgroups of the fused product, at most
// Point-per-lane product (recomputed blocks): a lane takes one point and
// loops over its observations; points with more observations than this are
// cut into pieces of at most this many (their sums go to split rows).
constexpr int kLaneObsMax = 16;

// Row of one cold observation outside its workgroup's window: its 9 camera
// values in the working precision; float64 rows are padded to whole 16-byte
// stores, float32 rows are not (36 bytes: every byte the product writes here
// is read back once by the camera sums).
template <typename S>
struct ColdRow;
template <>
struct ColdRow<double> {
  static constexpr int n = 10;
};
template <>
struct ColdRow<float> {
  static constexpr int n = 9;
};

// Camera rows of the recomputed-block product: the rotation as a unit
// quaternion (w, x, y, z), t, f, k1, k2, then the camera's 9 values of the
// product's input p and one pad (80 bytes in float32, 160 in float64).
constexpr int kProdCamRow = 20;
constexpr int kProdCamP = 10;  // offset of p in the row

// Camera row of the product's input vector p with stored blocks: its 9 values
// padded to 10 doubles (5 x 16 B) or 16 floats (64 B, gathered by quads of
// lanes).
template <typename S>
struct CamPad;
template <>
struct CamPad<double> {
  static constexpr int n = 10;
};
template <>
struct CamPad<float> {
  static constexpr int n = 16;
};

// Wave tile: a run of whole points (or one slice of a point with more than
// kTileMax observations) covering <= kTileMax consecutive observations.
struct Tile {
  int obs_begin;   // first observation (internal order)
  int pt_begin;    // first point (internal order)
  int cold_begin;  // first row in the cold-camera row buffer
  int split_row;   // row in the split-point buffer, -1 for ordinary tiles
  int info;        // n_obs | n_pts << 7 | seg_steps << 14 | split << 17 | first slice << 18
  int pad0, pad1, pad2;
};
static_assert(sizeof(Tile) == 32, "tile is two dwordx4");

__host__ __device__ inline int tile_nobs(int info) { return info & 127; }
__host__ __device__ inline int tile_npts(int info) { return (info >> 7) & 127; }
__host__ __device__ inline int tile_steps(int info) { return (info >> 14) & 7; }
__host__ __device__ inline bool tile_split(int info) { return (info >> 17) & 1; }
__host__ __device__ inline bool tile_first(int info) { return (info >> 18) & 1; }

// Camera-major linearisation chunk: entries [begin, end) of camera cam, summed
// into output row `row`.
struct Chunk {
  int cam, begin, end, row;
};

// Points observed more than kTileMax times: their tiles' partial rows.
// A pose between-factor in internal camera ids: measured relative pose
// (Z_R row-major, Z_t) and the square-root weights of its rotation and
// translation rows.  128 bytes.
struct BetweenFactor {
  int ci, cj;
  double ZR[9];
  double Zt[3];
  double s_rot, s_trans;
  double pad;
};

struct SplitPoint {
  int pt, row_begin, nrows, pad;
};

// PCG / reduction scalars living on the device.
struct DevScalars {
  double pAp, alpha, rho, rr, bb, tol2, beta, pad0;
  int iter, done, reason, max_iter;
  // reduction results: [0] linearisation cost sum, [1] trial cost sum, [2] dot,
  // [3] absmax, [4..6] predicted-decrease dots, [7] between-factor r.r
  double red[8];
  int err;
  int last_x;  // the iteration that set `done` made a valid update whose x step is still due
  unsigned ticket;  // workgroups of the PCG update done so far (its last one sets the scalars)
  int pad1;
};
enum { PCG_RUNNING = 0, PCG_CONVERGED = 1, PCG_BREAKDOWN = 2, PCG_MAXITER = 3, PCG_ZERO_RHS = 4 };

// ---------------------------------------------------------------------------
// The handle.
// ---------------------------------------------------------------------------
struct Vectors {
  void* g;  // gradient J^T r
  void* D;  // damping diagonal
  void* x;
  void* r;
  void* z;
  void* p;
  void* w;
  void* v;  // scratch vector (hooks, adjoint right-hand side)
};

}  // namespace cba

struct caspar_ba {
  ~caspar_ba();
  int nc = 0, np = 0;
  int no = 0;
  int prec = CASPAR_FP64;
  int loss = CASPAR_LOSS_TRIVIAL;  // robust loss of the squared residual norm
  double loss_c = 1.0;             // its scale (pixels)
  bool rj = false;        // Jacobian recomputed in every product instead of stored
  int N = 0;              // 9 nc + 3 np
  hipStream_t stream = nullptr;
  int device = 0;

  // layout
  int K = 0;              // cameras accumulated in LDS (internal ids < K)
  int G = 0;              // workgroups of the fused product
  int n_tiles = 0;
  int n_cold = 0;         // observations of cameras >= K
  int n_cold_rows = 0;    // rows of the fused product for cameras >= K: one per observation outside
                          // its workgroup's window (working precision), then L per workgroup for the
                          // windows (float64, in win_rows)
  int L = 0;              // cold cameras in each workgroup's LDS window
  int cold_local_base = 0;  // first window row
  int n_split_tiles = 0;
  int n_split_pts = 0;
  int n_orphan_pts = 0;   // points without observations (internal ids [0, n_orphan))
  int n_chunks = 0;
  bool mv_small = false;  // the point-per-lane product runs four-wave workgroups
  int n_big_chunks = 0;  // chunks [0, n_big_chunks) take a workgroup each, the rest a wave
  int no_pad = 0;         // observations rounded up to the Jacobian block

  // parameters (float64, internal order)
  double* cam = nullptr;        // [nc][16]
  double* cam_trial = nullptr;
  void* cam_s = nullptr;        // [nc][16] camera rows in the working precision (linearisation, products)
  void* cam_trial_s = nullptr;  // [nc][16] trial camera rows in float32 (trial cost of the mixed form)
  void* pts_s = nullptr;        // points in the working precision: float32 [np][4], or X itself in float64
  void* wts = nullptr;          // [no] IRLS weights rho'(|r|^2) of the last linearisation (robust losses)
  double* X = nullptr;          // [np][3]
  double* X_trial = nullptr;

  // permutations
  int* cam_c2i = nullptr;
  int* cam_i2c = nullptr;
  int* pt_c2i = nullptr;
  int* pt_i2c = nullptr;
  int* obs_s2c = nullptr;       // internal observation -> caller index

  // point-major observation data
  uint32_t* meta = nullptr;     // cam | local point << 25
  double* px = nullptr;         // [no][2]
  void* J = nullptr;            // 12 columns x 2 rows, 16-byte chunks, chunk-major
  cba::Tile* tiles = nullptr;

  // camera-major data
  int* cm_obs = nullptr;        // [no] internal observation of each camera-major entry
  int* cm_pt = nullptr;         // [no] internal point of each camera-major entry
  double* cm_px = nullptr;      // [no][2] camera-major observed pixels (float64 form only)
  void* px_s = nullptr;         // [no][2] float32 copy of px (float32-mixed form)
  void* cm_px_s = nullptr;      // [no][2] the same in float32 (float32-mixed form only)
  int* cam_off = nullptr;       // [nc + 1]
  cba::Chunk* chunks = nullptr;
  int* chunk_off = nullptr;     // [nc + 1] chunks of camera c
  double* chunk_rows = nullptr; // [n_chunks][54]

  // fused product side buffers
  int* cold_lo = nullptr;       // [G] first camera of each product workgroup's LDS window
  void* p_cam = nullptr;        // camera rows of the product's input: [nc][CamPad] (stored blocks) or
                                // [nc][kProdCamRow] with the camera parameters (recomputed blocks)
  int* cold_list = nullptr;     // cold rows grouped by camera
  int* cold_off = nullptr;      // [nc - K + 1]
  void* cold_rows = nullptr;    // [cold_local_base][ColdRow<S>::n] rows of single cold observations
  double* win_rows = nullptr;   // [G][L][kColdRow] window sums (float64), inside the cold_rows region
  cba::SplitPoint* split_pts = nullptr;
  double* split_rows = nullptr; // [n_split_tiles][9]

  // point-per-lane product (recomputed blocks): lane units in internal point
  // order, 64 per wave tile; a unit is a whole point or a piece of at most
  // kLaneObsMax observations of a point with more
  int n_units = 0;
  int n_lane_tiles = 0;
  int n_lane_split_pts = 0;      // points cut into pieces
  int* unit_obs = nullptr;       // [n_units + 1] first observation of each unit
  int* unit_pt = nullptr;        // [n_units] point | piece << 31 | first piece << 30
  int* unit_row = nullptr;       // [n_units] split row of a piece (-1 for whole points)
  int2* lane_tiles = nullptr;    // [n_lane_tiles] (trip count, first cold row)
  int* lane_base = nullptr;      // [n_lane_tiles + 1] first step of each lane tile (sums of trip counts)
  uint32_t* lane_meta = nullptr; // recomputed blocks: the meta word lane l of lane tile t reads at its step i,
                                 // at (lane_base[t] + i) * 64 + l (coalesced per step)
  void* lane_wts = nullptr;      // recomputed blocks, robust loss: the IRLS weights in the same step order
  cba::SplitPoint* lane_split_pts = nullptr;
  double* lane_split_rows = nullptr;  // [pieces][kPtRowWidth] (3 used)
  void* hot_rows = nullptr;     // [G][K][9] per-workgroup hot-camera sums, working precision

  // normal-equation blocks
  double* Hcc = nullptr;        // [nc][45]
  double* Hpp = nullptr;        // [np][6]
  void* Mc = nullptr;           // [nc][45] inverse blocks (precision)
  void* Mp = nullptr;           // [np][6]
  cba::Vectors vec;

  // pose between-factors (in the caller's second workspace, set_between)
  int n_between = 0;
  cba::BetweenFactor* between = nullptr;  // [n_between]
  int* bt_off = nullptr;        // [nc + 1] incident factors of each internal camera
  int* bt_inc = nullptr;        // [2 n_between] factor * 2 + side (0: first camera, 1: second)
  double* bt_rows = nullptr;    // [nc][6] between part of the product's camera rows
  double* bt_blocks = nullptr;  // [n_between][kBetweenBlock] blocks at the last linearisation

  double* partials = nullptr;   // [kMaxPartials][4]
  double* gauge_rows = nullptr; // [256][35] gauge-projection partial sums
  cba::DevScalars* scal = nullptr;
  cba::DevScalars* scal_host = nullptr;  // pinned host memory the scalar read-backs land in
  // Mapped (coherent) read-back: a kernel stores the scalars into scal_host
  // and then publishes scal_seq at *scal_flag; the host polls the flag
  // instead of waiting for a copy engine and a stream synchronisation.
  // Null for a handle on the static workspace (which allocates nothing).
  unsigned* scal_flag = nullptr;
  char* scal_mapped_dev = nullptr;  // the device's address of the pinned block (struct, then flag)
  unsigned scal_seq = 0;
  cba::DevScalars scal_local{};          // their landing place for a handle on the static workspace
  int static_dev = -1;                   // device whose static workspace this handle holds (-1: none)

  // kernel timing (roofline reporting): every timing_every-th launch of the
  // fused product (counted over the launches since timing was switched on)
  // gets a pair of events; 0 is off
  int timing_every = 0;
  int64_t mv_seq = 0;           // product launches since timing was switched on
  int mv_in_solve = 0;          // product launches since the last harvest
  std::vector<hipEvent_t> ev_start, ev_stop;
  std::vector<int> ev_pos;      // mv_in_solve of each timed launch
  int ev_used = 0;
  int64_t mv_launches = 0;
  double mv_ms = 0.0;

  // state
  bool linearized = false;      // J, g, D, H match the current parameters
  double cost = 0.0;            // F at the current parameters (valid if linearized)
  double gmax = 0.0;
  double bj_lambda = -1.0;      // lambda of the stored block-Jacobi inverse
};

namespace cba {

// Arena planning: byte offsets of every region inside the caller workspace.
struct Plan {
  size_t total = 0;
  struct Region {
    size_t off = 0, bytes = 0;
  };
  Region cam, cam_trial, cam_s, cam_trial_s, pts_s, wts, px_s, cm_px_s, X, X_trial, cam_c2i, cam_i2c, pt_c2i, pt_i2c, obs_s2c, meta, px, J,
      tiles, cold_lo, p_cam, cm_obs, cm_pt, cm_px, cam_off, chunks, chunk_off, chunk_rows, cold_list, cold_off, cold_rows,
      split_pts, split_rows, hot_rows, Hcc, Hpp, Mc, Mp, vecs, partials, scal, gauge_rows, unit_obs, unit_pt,
      unit_row, lane_tiles, lane_split_pts, lane_split_rows, lane_base, lane_meta, lane_wts;
  size_t vec_bytes = 0;
  int K = 0, G = 0;
  size_t max_tiles = 0, max_chunks = 0, max_cold = 0, max_split_tiles = 0, max_split_pts = 0;
  size_t max_units = 0, max_lane_tiles = 0, max_pieces = 0, max_lane_split_pts = 0;
};
bool make_plan(int nc, int np, int64_t no, int mode, Plan& plan);

// The static workspace of caspar_ba_create_static (one per device, for
// callers that cannot allocate): its size, and the claim a handle holds on
// the current device's copy while it lives.
constexpr size_t kStaticWorkspaceBytes = (size_t)256 << 20;
void* static_workspace_claim(int dev);
void static_workspace_release(int dev);

inline size_t scalar_bytes(int prec) { return prec == CASPAR_FP64 ? 8 : 4; }

// IRLS weights for a kernel: null with the trivial loss.
template <typename S>
inline const S* weights_of(const caspar_ba* h) {
  return h->loss == CASPAR_LOSS_TRIVIAL ? nullptr : static_cast<const S*>(h->wts);
}
// The same in the point-per-lane product's step order (recomputed blocks).
template <typename S>
inline const S* lane_weights_of(const caspar_ba* h) {
  return h->loss == CASPAR_LOSS_TRIVIAL ? nullptr : static_cast<const S*>(h->lane_wts);
}

// Layout of the product's camera rows of p: stride of a row and offset of
// the camera's 9 values in it.
template <typename S>
inline int cam_row_stride(const caspar_ba* h) {
  return h->rj ? kProdCamRow : CamPad<S>::n;
}
inline int cam_row_p_off(const caspar_ba* h) { return h->rj ? kProdCamP : 0; }

// Observed pixels in the working precision (the float32 kernels use them
// only as float32): point-major and camera-major.
template <typename S>
inline const S* pixels_of(const caspar_ba* h) {
  return static_cast<const S*>(sizeof(S) == 4 ? h->px_s : static_cast<const void*>(h->px));
}
template <typename S>
inline const S* cm_pixels_of(const caspar_ba* h) {
  return static_cast<const S*>(sizeof(S) == 4 ? h->cm_px_s : static_cast<const void*>(h->cm_px));
}
template <typename S>
struct Pair;
template <>
struct Pair<float> {
  using type = float2;
};
template <>
struct Pair<double> {
  using type = double2;
};

// Points in the working precision: the float32 copy written at each
// linearisation, or the (current) float64 master rows.
inline const void* pts_table(const caspar_ba* h) {
  return h->prec == CASPAR_FP64 ? static_cast<const void*>(h->X) : h->pts_s;
}


// LDS of one fused-product workgroup: float64 sums of the K hot cameras,
// kPrivCopies private copies of the most observed ones, and the L cameras of
// the workgroup's cold window.
inline size_t matvec_lds_bytes(int K, int L) {
  const int P = K < kPrivCams ? K : kPrivCams;
  return ((size_t)K + (size_t)kPrivCopies * P + (size_t)L) * 9 * sizeof(double);
}
// the largest case, with the kernels' own reduction slots (16 doubles), fits
// the 160 KiB of LDS a workgroup can have on gfx950
static_assert(((size_t)kMaxHot + (size_t)kPrivCopies * kPrivCams + kColdWin) * 9 * sizeof(double) + 16 * 8 <=
                  160 * 1024,
              "product LDS exceeds 160 KiB");

// Launch helpers implemented per translation unit (S = double or float).
// layout.hip
void upload_cameras_bal(caspar_ba* h, const double* cams_bal_caller, double* cam_internal);
void upload_points(caspar_ba* h, const double* pts_caller, double* X_internal);
// linearize.hip
void run_linearize(caspar_ba* h);                   // J, g, H, D, cost, gmax
void launch_lane_weights(caspar_ba* h);             // IRLS weights into the product's step order
double run_cost(caspar_ba* h, const double* cam, const double* X, bool fp64);  // F at params
void launch_cost(caspar_ba* h, const double* cam, const double* X, bool fp64);  // its sums, no read-back
double cost_of(const caspar_ba* h, const DevScalars& s);  // F from the sums launch_cost left
void run_retract(caspar_ba* h, const void* delta);  // trial = current (+) delta
void run_export_linearization(caspar_ba* h, double* resid, double* jc, double* jp);
// matvec.hip
void run_matvec(caspar_ba* h, double lambda, const void* p, void* w, bool pcg_mode, bool pad_cams = true);
// pcg.hip
void run_block_jacobi(caspar_ba* h, double lambda);
void run_bj_apply(caspar_ba* h, const void* r, void* z);
int run_pcg(caspar_ba* h, double lambda, const void* b, bool negate_b, double tol, int max_iters,
            int check_every, void* x, double* rel_resid, int first_batch = 0);  // first poll after
                                                                              // max(check_every, first_batch)
double run_dot(caspar_ba* h, const void* a, const void* b, const void* wdiag);  // sum a b (w)
void run_pred_dots(caspar_ba* h, double* gx, double* xr, double* xDx);  // g^T x, x^T r, x^T D x
void launch_pred_dots(caspar_ba* h);                // the same into red[4..6], no read-back
void pred_dots_of(const caspar_ba* h, const DevScalars& s, double* gx, double* xr, double* xDx);
double run_absmax(caspar_ba* h, const void* a);
void launch_absmax(caspar_ba* h, const void* a);    // max |a| into red[3], no read-back
void run_to_caller_vector(caspar_ba* h, const void* internal, double* caller);
void run_from_caller_vector(caspar_ba* h, const double* caller, void* internal);
void run_zero(caspar_ba* h, void* v, size_t count_scalars);
void timing_events(caspar_ba* h, hipEvent_t* start, hipEvent_t* stop);  // null pair when timing is off
void timing_harvest(caspar_ba* h, int effective);  // after a sync: count timed launches among the first `effective`
double matvec_algorithmic_bytes(const caspar_ba* h);
// between.hip
void run_between_lin(caspar_ba* h);                 // adds g, H_cc, D terms; cost sum r.r into red[7]
double run_between_cost(caspar_ba* h, const double* cam);  // 1/2 sum |r|^2 at camera rows `cam`
void launch_between_cost(caspar_ba* h, const double* cam);  // its sum r.r into red[7], no read-back
void run_between_product(caspar_ba* h, const void* p, bool pcg_mode);  // bt_rows and pAp partials
unsigned between_grid(const caspar_ba* h);          // workgroups of the per-camera between kernels
int matvec_waves(int prec, bool rj);  // waves per workgroup of the fused product
int matvec_small_waves();              // the same, point-per-lane product on a small problem
// helpers
void sync(caspar_ba* h);
DevScalars read_scalars(caspar_ba* h);

}  // namespace cba

// ---------------------------------------------------------------------------
// Device helpers.
// ---------------------------------------------------------------------------
namespace cba {

template <typename T>
struct Scalar;
template <>
struct Scalar<double> {
  static constexpr double eps() { return 10.0 * 2.220446049250313e-16; }
};
template <>
struct Scalar<float> {
  static constexpr float eps() { return 10.0f * 1.1920928955078125e-07f; }
};

// Index of (k, l), k <= l, in the row-major upper triangle of a 9x9 block.
__host__ __device__ constexpr int tri9(int k, int l) { return k * 9 - k * (k - 1) / 2 + (l - k); }

__device__ inline double clamp_diag(double d) { return fmin(fmax(d, 1e-6), 1e32); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// Sum over the workgroup; every thread gets the result.  `lds` holds one
// double per wave.  Contains barriers: call from all threads.
__device__ inline double block_sum(double v, double* lds) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += lds[i];
  return s;
}

__device__ inline double block_max(double v, double* lds) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s = fmax(s, lds[i]);
  return s;
}

}  // namespace cba
