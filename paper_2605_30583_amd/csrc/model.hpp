// Device-side camera model: the Snavely reprojection factor of the paper's
// Section VI-A and its tangent-space Jacobian (Section V), plus the SO(3)
// exponential, logarithm and inverse right Jacobian used at the boundary.
#pragma once

#include "common.hpp"

namespace cba {

// Camera in registers, converted to the working precision T.
template <typename T>
struct Cam {
  T R[9];  // row-major
  T t[3];
  T f, k1, k2;
};

// Robust loss of the squared residual norm s with scale c: returns rho(s)
// and sets w = rho'(s), the IRLS weight.  kind: CASPAR_LOSS_TRIVIAL (rho = s),
// CASPAR_LOSS_HUBER (s inside c^2, 2 c sqrt(s) - c^2 outside),
// CASPAR_LOSS_CAUCHY (c^2 log(1 + s / c^2)).
__device__ inline double robust_rho(int kind, double c, double s, double& w) {
  const double c2 = c * c;
  if (kind == CASPAR_LOSS_HUBER) {
    if (s <= c2) {
      w = 1.0;
      return s;
    }
    const double rs = sqrt(s);
    w = c / rs;
    return 2.0 * c * rs - c2;
  }
  if (kind == CASPAR_LOSS_CAUCHY) {
    w = 1.0 / (1.0 + s / c2);
    return c2 * log1p(s / c2);
  }
  w = 1.0;
  return s;
}

// Point coordinates in the working precision: float32 rows (x, y, z, 0) read
// with one 16-byte load, or the float64 master rows of 3.
template <typename S>
__device__ inline void load_point(const S* __restrict__ tab, size_t i, S (&x)[3]);
template <>
__device__ inline void load_point<float>(const float* __restrict__ tab, size_t i, float (&x)[3]) {
  const float4 v = reinterpret_cast<const float4*>(tab)[i];
  x[0] = v.x;
  x[1] = v.y;
  x[2] = v.z;
}
template <>
__device__ inline void load_point<double>(const double* __restrict__ tab, size_t i, double (&x)[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) x[k] = tab[3 * i + k];
}

// Loads one 16-double camera row [R(9) t(3) f k1 k2 pad] (128-byte aligned).
template <typename T>
__device__ inline Cam<T> load_cam(const double* __restrict__ camtab, int c) {
  const double2* row = reinterpret_cast<const double2*>(camtab + (size_t)c * kCamStride);
  double v[16];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double2 q = row[i];
    v[2 * i] = q.x;
    v[2 * i + 1] = q.y;
  }
  Cam<T> cam;
#pragma unroll
  for (int i = 0; i < 9; ++i) cam.R[i] = (T)v[i];
  cam.t[0] = (T)v[9];
  cam.t[1] = (T)v[10];
  cam.t[2] = (T)v[11];
  cam.f = (T)v[12];
  cam.k1 = (T)v[13];
  cam.k2 = (T)v[14];
  return cam;
}

// Quad-cooperative gather of 64-byte float32 rows (16 floats, the table
// 64-byte aligned).  Gathering a row per lane takes four 16-byte requests,
// each lane of each request at its own row; here request i fetches, for every
// quad of lanes, the row of the quad's lane i, lane j of the quad taking
// quarter j, so that a request touches one row per quad instead of one per
// lane.  quad_rows_take() then transposes the 4 x 4 quarters within the quad
// (two rounds of lane swaps), leaving each lane its own row.  Both must run
// with all lanes of the wave active, and the workgroup size must be a
// multiple of 64.
struct QuadRows {
  float4 q[4];
};

__device__ inline void quad_rows_request(const float* __restrict__ tab, int row, QuadRows& r) {
  const float4* t4 = reinterpret_cast<const float4*>(tab) + (threadIdx.x & 3u);
  // quad_perm broadcasts of quad lanes 0..3
  const int r0 = __builtin_amdgcn_mov_dpp(row, 0x00, 0xf, 0xf, false);
  const int r1 = __builtin_amdgcn_mov_dpp(row, 0x55, 0xf, 0xf, false);
  const int r2 = __builtin_amdgcn_mov_dpp(row, 0xaa, 0xf, 0xf, false);
  const int r3 = __builtin_amdgcn_mov_dpp(row, 0xff, 0xf, 0xf, false);
  r.q[0] = t4[4 * (size_t)r0];
  r.q[1] = t4[4 * (size_t)r1];
  r.q[2] = t4[4 * (size_t)r2];
  r.q[3] = t4[4 * (size_t)r3];
}

// One dword plane of the in-quad 4 x 4 transpose: lane j holds a_i = M[j][i]
// and ends with a_i = M[i][j].  Round one swaps with lane j ^ 1 (pairs
// (a0, a1), (a2, a3)), round two with lane j ^ 2 (pairs (a0, a2), (a1, a3)).
__device__ inline float quad_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xb1, 0xf, 0xf, false));
}
__device__ inline float quad_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4e, 0xf, 0xf, false));
}
__device__ inline void quad_swap(float& lo, float& hi, bool upper, bool two) {
  const float s = upper ? lo : hi;
  const float r = two ? quad_xor2(s) : quad_xor1(s);
  lo = upper ? r : lo;
  hi = upper ? hi : r;
}
__device__ inline void quad_transpose(float& a0, float& a1, float& a2, float& a3, bool b0, bool b1) {
  quad_swap(a0, a1, b0, false);
  quad_swap(a2, a3, b0, false);
  quad_swap(a0, a2, b1, true);
  quad_swap(a1, a3, b1, true);
}

__device__ inline void quad_rows_take(QuadRows& r, float (&v)[16]) {
  const bool b0 = (threadIdx.x & 1u) != 0u, b1 = (threadIdx.x & 2u) != 0u;
  quad_transpose(r.q[0].x, r.q[1].x, r.q[2].x, r.q[3].x, b0, b1);
  quad_transpose(r.q[0].y, r.q[1].y, r.q[2].y, r.q[3].y, b0, b1);
  quad_transpose(r.q[0].z, r.q[1].z, r.q[2].z, r.q[3].z, b0, b1);
  quad_transpose(r.q[0].w, r.q[1].w, r.q[2].w, r.q[3].w, b0, b1);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[4 * i] = r.q[i].x;
    v[4 * i + 1] = r.q[i].y;
    v[4 * i + 2] = r.q[i].z;
    v[4 * i + 3] = r.q[i].w;
  }
}

// A camera row of the working-precision table (16 values: R t f k1 k2 pad)
// in two halves: cam_request() issues the loads (float32: quad-cooperative,
// all lanes active), cam_take() turns what arrived into a camera (float32:
// the in-quad transpose, all lanes active).
template <typename T>
struct CamReq;
template <>
struct CamReq<float> {
  QuadRows r;
};
template <>
struct CamReq<double> {
  Cam<double> c;
};
template <typename T>
__device__ inline void cam_request(const T* __restrict__ tab, int c, CamReq<T>& q);
template <>
__device__ inline void cam_request<double>(const double* __restrict__ tab, int c, CamReq<double>& q) {
  q.c = load_cam<double>(tab, c);
}
template <>
__device__ inline void cam_request<float>(const float* __restrict__ tab, int c, CamReq<float>& q) {
  static_assert(kCamStride == 16, "64-byte float32 camera rows");
  quad_rows_request(tab, c, q.r);
}
template <typename T>
__device__ inline Cam<T> cam_take(CamReq<T>& q);
template <>
__device__ inline Cam<double> cam_take<double>(CamReq<double>& q) {
  return q.c;
}
template <>
__device__ inline Cam<float> cam_take<float>(CamReq<float>& q) {
  float v[16];
  quad_rows_take(q.r, v);
  Cam<float> cam;
#pragma unroll
  for (int i = 0; i < 9; ++i) cam.R[i] = v[i];
  cam.t[0] = v[9];
  cam.t[1] = v[10];
  cam.t[2] = v[11];
  cam.f = v[12];
  cam.k1 = v[13];
  cam.k2 = v[14];
  return cam;
}

// Camera row of the working-precision table (16 values: R t f k1 k2 pad),
// read with 16-byte vector loads, one row per lane.
template <typename T>
__device__ inline Cam<T> load_cam_s(const T* __restrict__ tab, int c);
template <>
__device__ inline Cam<double> load_cam_s<double>(const double* __restrict__ tab, int c) {
  return load_cam<double>(tab, c);
}
template <>
__device__ inline Cam<float> load_cam_s<float>(const float* __restrict__ tab, int c) {
  const float4* row = reinterpret_cast<const float4*>(tab + (size_t)c * kCamStride);
  float v[16];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float4 q = row[i];
    v[4 * i] = q.x;
    v[4 * i + 1] = q.y;
    v[4 * i + 2] = q.z;
    v[4 * i + 3] = q.w;
  }
  Cam<float> cam;
#pragma unroll
  for (int i = 0; i < 9; ++i) cam.R[i] = v[i];
  cam.t[0] = v[9];
  cam.t[1] = v[10];
  cam.t[2] = v[11];
  cam.f = v[12];
  cam.k1 = v[13];
  cam.k2 = v[14];
  return cam;
}

// One camera row of the recomputed-block product (kProdCamRow values) with
// 16-byte vector loads.
template <typename S>
__device__ inline void load_prod_cam(const S* __restrict__ tab, int c, S (&row)[kProdCamRow]);
template <>
__device__ inline void load_prod_cam<float>(const float* __restrict__ tab, int c, float (&row)[kProdCamRow]) {
  const float4* r = reinterpret_cast<const float4*>(tab + (size_t)c * kProdCamRow);
#pragma unroll
  for (int i = 0; i < kProdCamRow / 4; ++i) {
    const float4 v = r[i];
    row[4 * i] = v.x;
    row[4 * i + 1] = v.y;
    row[4 * i + 2] = v.z;
    row[4 * i + 3] = v.w;
  }
}
template <>
__device__ inline void load_prod_cam<double>(const double* __restrict__ tab, int c, double (&row)[kProdCamRow]) {
  const double2* r = reinterpret_cast<const double2*>(tab + (size_t)c * kProdCamRow);
#pragma unroll
  for (int i = 0; i < kProdCamRow / 2; ++i) {
    const double2 v = r[i];
    row[2 * i] = v.x;
    row[2 * i + 1] = v.y;
  }
}

// Camera of a product row: R from the unit quaternion (w, x, y, z),
//   R = I + 2 w [v]x + 2 [v]x^2,  v = (x, y, z).
template <typename T>
__device__ inline Cam<T> prod_cam(const T (&row)[kProdCamRow]) {
  const T w = row[0], x = row[1], y = row[2], z = row[3];
  const T x2 = x + x, y2 = y + y, z2 = z + z;
  const T xx = x * x2, yy = y * y2, zz = z * z2;
  const T xy = x * y2, xz = x * z2, yz = y * z2;
  const T wx = w * x2, wy = w * y2, wz = w * z2;
  Cam<T> c;
  c.R[0] = (T)1 - (yy + zz);
  c.R[1] = xy - wz;
  c.R[2] = xz + wy;
  c.R[3] = xy + wz;
  c.R[4] = (T)1 - (xx + zz);
  c.R[5] = yz - wx;
  c.R[6] = xz - wy;
  c.R[7] = yz + wx;
  c.R[8] = (T)1 - (xx + yy);
  c.t[0] = row[4];
  c.t[1] = row[5];
  c.t[2] = row[6];
  c.f = row[7];
  c.k1 = row[8];
  c.k2 = row[9];
  return c;
}

// Residual of one observation.  P = R X + t; the depth keeps its sign away
// from zero (d + eps sign(d), sign(0) = +1); p = -P_xy / d;
// radial = 1 + k1 |p|^2 + k2 |p|^4; r = f radial p - px.
template <typename T>
__device__ inline void snavely_residual(const Cam<T>& c, T X0, T X1, T X2, T px0, T px1, T& r0,
                                        T& r1) {
  const T P0 = fma(c.R[0], X0, fma(c.R[1], X1, fma(c.R[2], X2, c.t[0])));
  const T P1 = fma(c.R[3], X0, fma(c.R[4], X1, fma(c.R[5], X2, c.t[1])));
  const T P2 = fma(c.R[6], X0, fma(c.R[7], X1, fma(c.R[8], X2, c.t[2])));
  const T d = P2 + (P2 >= (T)0 ? Scalar<T>::eps() : -Scalar<T>::eps());
  const T id = (T)1 / d;
  const T p0 = -P0 * id, p1 = -P1 * id;
  const T n2 = fma(p0, p0, p1 * p1);
  const T rad = fma(n2, fma(c.k2, n2, c.k1), (T)1);
  const T fr = c.f * rad;
  r0 = fma(fr, p0, -px0);
  r1 = fma(fr, p1, -px1);
}

// Residual and Jacobian columns.  col[j] = (J[0][j], J[1][j]) for the 12
// columns [dw(3), dt(3), df, dk1, dk2, dX(3)].
//   du/dp = f (radial I + 2 (k1 + 2 k2 |p|^2) p p^T) =: A
//   dp/dP = -(1/d) [I | p]          => B = du/dP = -(1/d) [A | A p]
//   dP/dt = I, dP/dX = R, dP/dw = -R [X]x (right perturbation)
//   J_t = B, J_X = B R, row i of J_w = X x (row i of J_X)
//   J_f = radial p, J_k1 = f |p|^2 p, J_k2 = f |p|^4 p.
template <typename T>
__device__ inline void snavely_jacobian(const Cam<T>& c, T X0, T X1, T X2, T px0, T px1, T& r0,
                                        T& r1, T col[12][2]) {
  const T P0 = fma(c.R[0], X0, fma(c.R[1], X1, fma(c.R[2], X2, c.t[0])));
  const T P1 = fma(c.R[3], X0, fma(c.R[4], X1, fma(c.R[5], X2, c.t[1])));
  const T P2 = fma(c.R[6], X0, fma(c.R[7], X1, fma(c.R[8], X2, c.t[2])));
  const T d = P2 + (P2 >= (T)0 ? Scalar<T>::eps() : -Scalar<T>::eps());
  const T id = (T)1 / d;
  const T p0 = -P0 * id, p1 = -P1 * id;
  const T n2 = fma(p0, p0, p1 * p1);
  const T rad = fma(n2, fma(c.k2, n2, c.k1), (T)1);
  const T fr = c.f * rad;
  r0 = fma(fr, p0, -px0);
  r1 = fma(fr, p1, -px1);

  const T fs = c.f * (T)2 * fma((T)2 * c.k2, n2, c.k1);
  const T a00 = fma(fs * p0, p0, fr);
  const T a01 = fs * p0 * p1;
  const T a11 = fma(fs * p1, p1, fr);
  const T m = -id;
  const T B00 = m * a00, B01 = m * a01, B10 = m * a01, B11 = m * a11;
  const T B02 = fma(B00, p0, B01 * p1);
  const T B12 = fma(B10, p0, B11 * p1);
  // J_X = B R
  T Jx0[3], Jx1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Jx0[k] = fma(B00, c.R[k], fma(B01, c.R[3 + k], B02 * c.R[6 + k]));
    Jx1[k] = fma(B10, c.R[k], fma(B11, c.R[3 + k], B12 * c.R[6 + k]));
  }
  // J_w rows: X x J_X rows
  col[0][0] = fma(X1, Jx0[2], -X2 * Jx0[1]);
  col[1][0] = fma(X2, Jx0[0], -X0 * Jx0[2]);
  col[2][0] = fma(X0, Jx0[1], -X1 * Jx0[0]);
  col[0][1] = fma(X1, Jx1[2], -X2 * Jx1[1]);
  col[1][1] = fma(X2, Jx1[0], -X0 * Jx1[2]);
  col[2][1] = fma(X0, Jx1[1], -X1 * Jx1[0]);
  col[3][0] = B00;
  col[3][1] = B10;
  col[4][0] = B01;
  col[4][1] = B11;
  col[5][0] = B02;
  col[5][1] = B12;
  col[6][0] = rad * p0;
  col[6][1] = rad * p1;
  const T fn2 = c.f * n2;
  col[7][0] = fn2 * p0;
  col[7][1] = fn2 * p1;
  col[8][0] = fn2 * n2 * p0;
  col[8][1] = fn2 * n2 * p1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    col[9 + k][0] = Jx0[k];
    col[9 + k][1] = Jx1[k];
  }
}

// 1/d for the projection: the hardware reciprocal in float32 (within one ulp,
// below the rounding of the float32 products that use it), exact division in
// float64.
__device__ inline float proj_recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ inline double proj_recip(double d) { return 1.0 / d; }

// One observation's share of the normal-equation product, from the camera
// and the point, without forming its blocks.  With the block structure
// above (J_t = B, J_X = B R, row i of J_w = X x row i of J_X):
//   q        = J_c p_c + J_X p_X
//            = B (R (p_X + p_w x X) + p_t) + p (radial p_f + f |p|^2 (p_k1 + |p|^2 p_k2)),
// and with q~ = wgt q (the IRLS weight, 1 without a robust loss)
//   J_t^T q~ = B^T q~,   J_X^T q~ = R^T B^T q~,   J_w^T q~ = X x (J_X^T q~),
//   J_f,k1,k2^T q~ = (radial, f |p|^2, f |p|^4) (p . q~).
// pc holds the camera tangent [dw, dt, df, dk1, dk2]; returns q . q~ (the
// observation's term of p^T J^T W J p), yc (9) and yp (3) are J_c^T q~ and
// J_X^T q~.  WEIGHTED = false skips the weight (wgt is then ignored).
template <bool WEIGHTED, typename T>
__device__ inline T snavely_apply(const Cam<T>& c, T X0, T X1, T X2, const T* pc, const T pp[3], T wgt,
                                  T yc[9], T yp[3]) {
  const T P0 = fma(c.R[0], X0, fma(c.R[1], X1, fma(c.R[2], X2, c.t[0])));
  const T P1 = fma(c.R[3], X0, fma(c.R[4], X1, fma(c.R[5], X2, c.t[1])));
  const T P2 = fma(c.R[6], X0, fma(c.R[7], X1, fma(c.R[8], X2, c.t[2])));
  const T d = P2 + (P2 >= (T)0 ? Scalar<T>::eps() : -Scalar<T>::eps());
  const T m = -proj_recip(d);
  const T p0 = P0 * m, p1 = P1 * m;
  const T n2 = fma(p0, p0, p1 * p1);
  const T rad = fma(n2, fma(c.k2, n2, c.k1), (T)1);
  const T fr = c.f * rad;
  const T fs = c.f * (T)2 * fma((T)2 * c.k2, n2, c.k1);
  // B = m [A | A p], A = fr I + fs p p^T
  const T fp0 = fs * p0, fp1 = fs * p1;
  const T B00 = m * fma(fp0, p0, fr), B01 = m * (fp0 * p1), B11 = m * fma(fp1, p1, fr);
  const T B02 = fma(B00, p0, B01 * p1);
  const T B12 = fma(B01, p0, B11 * p1);
  // v = R (p_X + p_w x X) + p_t
  const T u0 = fma(pc[1], X2, fma(-pc[2], X1, pp[0]));
  const T u1 = fma(pc[2], X0, fma(-pc[0], X2, pp[1]));
  const T u2 = fma(pc[0], X1, fma(-pc[1], X0, pp[2]));
  const T v0 = fma(c.R[0], u0, fma(c.R[1], u1, fma(c.R[2], u2, pc[3])));
  const T v1 = fma(c.R[3], u0, fma(c.R[4], u1, fma(c.R[5], u2, pc[4])));
  const T v2 = fma(c.R[6], u0, fma(c.R[7], u1, fma(c.R[8], u2, pc[5])));
  const T fn2 = c.f * n2;
  const T s = fma(rad, pc[6], fn2 * fma(n2, pc[8], pc[7]));
  const T q0 = fma(B00, v0, fma(B01, v1, fma(B02, v2, p0 * s)));
  const T q1 = fma(B01, v0, fma(B11, v1, fma(B12, v2, p1 * s)));
  const T w0 = WEIGHTED ? wgt * q0 : q0, w1 = WEIGHTED ? wgt * q1 : q1;
  // transposes
  const T g0 = fma(B00, w0, B01 * w1);
  const T g1 = fma(B01, w0, B11 * w1);
  const T g2 = fma(B02, w0, B12 * w1);
  yp[0] = fma(c.R[0], g0, fma(c.R[3], g1, c.R[6] * g2));
  yp[1] = fma(c.R[1], g0, fma(c.R[4], g1, c.R[7] * g2));
  yp[2] = fma(c.R[2], g0, fma(c.R[5], g1, c.R[8] * g2));
  yc[0] = fma(X1, yp[2], -X2 * yp[1]);
  yc[1] = fma(X2, yp[0], -X0 * yp[2]);
  yc[2] = fma(X0, yp[1], -X1 * yp[0]);
  yc[3] = g0;
  yc[4] = g1;
  yc[5] = g2;
  const T h = fma(p0, w0, p1 * w1);
  yc[6] = rad * h;
  yc[7] = fn2 * h;
  yc[8] = fn2 * n2 * h;
  return fma(w0, q0, w1 * q1);
}

// Exp of an angle-axis vector (Rodrigues), row-major 3x3.
// R = I + s [w]x + c [w]x^2 with s = sin(a)/a, c = (1 - cos a)/a^2;
// series below a = 1e-4.
__device__ inline void so3_exp(double w0, double w1, double w2, double R[9]) {
  const double a2 = w0 * w0 + w1 * w1 + w2 * w2;
  double s, c;
  if (a2 < 1e-8) {
    s = 1.0 - a2 / 6.0 + a2 * a2 / 120.0;
    c = 0.5 - a2 / 24.0 + a2 * a2 / 720.0;
  } else {
    const double a = sqrt(a2);
    double sn, cs;
    sincos(a, &sn, &cs);
    s = sn / a;
    c = (1.0 - cs) / a2;
  }
  // [w]x^2 = w w^T - a2 I
  R[0] = 1.0 + c * (w0 * w0 - a2);
  R[1] = c * w0 * w1 - s * w2;
  R[2] = c * w0 * w2 + s * w1;
  R[3] = c * w1 * w0 + s * w2;
  R[4] = 1.0 + c * (w1 * w1 - a2);
  R[5] = c * w1 * w2 - s * w0;
  R[6] = c * w2 * w0 - s * w1;
  R[7] = c * w2 * w1 + s * w0;
  R[8] = 1.0 + c * (w2 * w2 - a2);
}

// Log of a rotation matrix as an angle-axis vector, through the unit
// quaternion (largest-component branch, accurate up to angle pi).
__device__ inline void so3_log(const double R[9], double w[3]) {
  const double tr = R[0] + R[4] + R[8];
  double q0, q1, q2, q3;  // w, x, y, z
  if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
    q0 = 0.5 * sqrt(fmax(0.0, 1.0 + tr));
    const double s = 0.25 / q0;
    q1 = (R[7] - R[5]) * s;
    q2 = (R[2] - R[6]) * s;
    q3 = (R[3] - R[1]) * s;
  } else if (R[0] >= R[4] && R[0] >= R[8]) {
    q1 = 0.5 * sqrt(fmax(0.0, 1.0 + R[0] - R[4] - R[8]));
    const double s = 0.25 / q1;
    q2 = (R[1] + R[3]) * s;
    q3 = (R[2] + R[6]) * s;
    q0 = (R[7] - R[5]) * s;
  } else if (R[4] >= R[8]) {
    q2 = 0.5 * sqrt(fmax(0.0, 1.0 + R[4] - R[0] - R[8]));
    const double s = 0.25 / q2;
    q1 = (R[1] + R[3]) * s;
    q3 = (R[5] + R[7]) * s;
    q0 = (R[2] - R[6]) * s;
  } else {
    q3 = 0.5 * sqrt(fmax(0.0, 1.0 + R[8] - R[0] - R[4]));
    const double s = 0.25 / q3;
    q1 = (R[2] + R[6]) * s;
    q2 = (R[5] + R[7]) * s;
    q0 = (R[3] - R[1]) * s;
  }
  if (q0 < 0.0) {
    q0 = -q0;
    q1 = -q1;
    q2 = -q2;
    q3 = -q3;
  }
  const double vn = sqrt(q1 * q1 + q2 * q2 + q3 * q3);
  double k;
  if (vn < 1e-12) {
    k = 2.0 / q0;  // angle ~ 2 vn / q0
  } else {
    k = 2.0 * atan2(vn, q0) / vn;
  }
  w[0] = k * q1;
  w[1] = k * q2;
  w[2] = k * q3;
}

// g_tangent = J_r^-1(w)^T g_aa, the gradient with respect to a right
// perturbation from the gradient with respect to the angle-axis vector.
// J_r^-1(w) = I + 1/2 [w]x + (1/a^2 - cot(a/2) / (2a)) [w]x^2.
__device__ inline void so3_grad_to_tangent(const double w[3], const double g[3], double out[3]) {
  const double a2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double c;
  if (a2 < 1e-6) {
    c = 1.0 / 12.0 + a2 / 720.0;
  } else {
    const double a = sqrt(a2);
    c = 1.0 / a2 - 1.0 / (2.0 * a * tan(0.5 * a));
  }
  // J^T g = g - 1/2 [w]x g + c [w]x^2 g   ([w]x^T = -[w]x, ([w]x^2)^T = [w]x^2)
  const double wxg0 = w[1] * g[2] - w[2] * g[1];
  const double wxg1 = w[2] * g[0] - w[0] * g[2];
  const double wxg2 = w[0] * g[1] - w[1] * g[0];
  const double wg = w[0] * g[0] + w[1] * g[1] + w[2] * g[2];
  // [w]x^2 g = w (w.g) - a2 g
  out[0] = g[0] - 0.5 * wxg0 + c * (w[0] * wg - a2 * g[0]);
  out[1] = g[1] - 0.5 * wxg1 + c * (w[1] * wg - a2 * g[1]);
  out[2] = g[2] - 0.5 * wxg2 + c * (w[2] * wg - a2 * g[2]);
}

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// Jacobian storage: blocked structure-of-arrays.  Observations are grouped
// in blocks of kJBlock; inside a block each 16-byte chunk (two Jacobian
// columns x two rows in float64, four columns in float32) is stored for all
// kJBlock observations before the next chunk:
//   chunk k of observation o lives at ((o / kJBlock) * kChunks + k) * kJBlock + o % kJBlock
// so a wave's 64 lanes read 1 KiB contiguous per chunk and a workgroup's
// consecutive tiles stream one contiguous region.
constexpr int kJBlock = 1024;

__device__ __host__ inline size_t jidx(int o, int k, int nchunks) {
  return ((size_t)(o / kJBlock) * nchunks + k) * kJBlock + (o % kJBlock);
}

template <typename S>
struct JStore;

// float64: 12 chunks, chunk j = column j (two rows).
template <>
struct JStore<double> {
  static constexpr int kChunks = 12;
  __device__ static void store(void* J, int o, const double col[12][2]) {
    double2* Jv = reinterpret_cast<double2*>(J);
#pragma unroll
    for (int j = 0; j < 12; ++j) Jv[jidx(o, j, kChunks)] = make_double2(col[j][0], col[j][1]);
  }
  __device__ static void load(const void* J, int o, double col[12][2]) {
    const dvec2* Jv = reinterpret_cast<const dvec2*>(J);
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      const dvec2 v = __builtin_nontemporal_load(&Jv[jidx(o, j, kChunks)]);
      col[j][0] = v.x;
      col[j][1] = v.y;
    }
  }
};

// float32: 6 chunks, chunk k = columns 2k, 2k+1 (two rows each).
template <>
struct JStore<float> {
  static constexpr int kChunks = 6;
  __device__ static void store(void* J, int o, const float col[12][2]) {
    float4* Jv = reinterpret_cast<float4*>(J);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      Jv[jidx(o, k, kChunks)] = make_float4(col[2 * k][0], col[2 * k][1], col[2 * k + 1][0], col[2 * k + 1][1]);
  }
  __device__ static void load(const void* J, int o, float col[12][2]) {
    const fvec4* Jv = reinterpret_cast<const fvec4*>(J);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const fvec4 v = __builtin_nontemporal_load(&Jv[jidx(o, k, kChunks)]);
      col[2 * k][0] = v.x;
      col[2 * k][1] = v.y;
      col[2 * k + 1][0] = v.z;
      col[2 * k + 1][1] = v.w;
    }
  }
};

// Jacobian columns of an observation, from the stored blocks or evaluated
// again from the working-precision camera row and the point (bitwise the
// values the linearisation produced).
template <typename S, bool RJ>
__device__ inline void jacobian_of(const void* J, const S* __restrict__ cam_s, const double* __restrict__ X,
                                   int o, int ci, int pi, S col[12][2]) {
  if (RJ) {
    const Cam<S> c = load_cam_s<S>(cam_s, ci);
    const double* Xp = X + 3 * (size_t)pi;
    S r0, r1;
    snavely_jacobian<S>(c, (S)Xp[0], (S)Xp[1], (S)Xp[2], (S)0, (S)0, r0, r1, col);
  } else {
    JStore<S>::load(J, o, col);
  }
}

}  // namespace cba
