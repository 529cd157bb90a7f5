// Plain FP64 CPU reference of the MP-weighted Gaussian-splatting path.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg load this library. It shares no code, header,
// table or helper with the GPU library and must never be used by it.
//
// What it computes (the paper only states that Gaussians contribute to pixel u
// with normalised weights omega during rasterisation, Sec. IV-D around
// Eq. (20), and that colour and depth are rendered from the pose, Eq. (21)-(22);
// the renderer below is the published EWA-splatting / 3DGS compositing model):
//   project : world mean -> camera (pose T_cw), 3D covariance from log-scale and
//             quaternion, Jacobian of the pinhole projection, 2D covariance
//             plus a 0.3 px^2 low-pass, its inverse (conic), pixel mean,
//             sigmoid opacity, and the opacity-aware support radius.
//   render  : per pixel, every kept Gaussian in ascending (depth, id) order,
//             alpha = min(0.99, o exp(-1/2 d^T conic d)), skip alpha < 1/255,
//             stop before adding a Gaussian that drops T below 1e-4.
//             C += a T c, D += a T z, M += a T m (M is the MP channel).
//   backward: plain reverse mode through render (every per-step value is
//             stored) and through the projection, to the Gaussian parameters
//             and the left-perturbation SE(3) twist (rho, phi) of the pose.
// Everything is evaluated in double precision.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

struct Cam {
  int W, H;
  double fx, fy, cx, cy, znear;
  double R[3][3];
  double t[3];
};

// cam: [W, H, fx, fy, cx, cy, z_near, T_cw (12, row-major 3x4)]
Cam read_cam(const double* c) {
  Cam k;
  k.W = (int)c[0];
  k.H = (int)c[1];
  k.fx = c[2]; k.fy = c[3]; k.cx = c[4]; k.cy = c[5]; k.znear = c[6];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) k.R[i][j] = c[7 + 4 * i + j];
    k.t[i] = c[7 + 4 * i + 3];
  }
  return k;
}

typedef double M3[3][3];

void matmul3(const M3 a, const M3 b, M3 out) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += a[i][k] * b[k][j];
      r[i][j] = s;
    }
  std::memcpy(out, r, sizeof(M3));
}

void transpose3(const M3 a, M3 out) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r[i][j] = a[j][i];
  std::memcpy(out, r, sizeof(M3));
}

// rotation matrix of a unit quaternion (w, x, y, z), Hamilton convention
void quat_to_rot(double w, double x, double y, double z, M3 R) {
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

// d R / d(w,x,y,z) for the formula above
void quat_rot_derivs(double w, double x, double y, double z, M3 dR[4]) {
  const double dw[3][3] = {{0, -2 * z, 2 * y}, {2 * z, 0, -2 * x}, {-2 * y, 2 * x, 0}};
  const double dx[3][3] = {{0, 2 * y, 2 * z}, {2 * y, -4 * x, -2 * w}, {2 * z, 2 * w, -4 * x}};
  const double dy[3][3] = {{-4 * y, 2 * x, 2 * w}, {2 * x, 0, 2 * z}, {-2 * w, 2 * z, -4 * y}};
  const double dz[3][3] = {{-4 * z, -2 * w, 2 * x}, {2 * w, -4 * z, 2 * y}, {2 * x, 2 * y, 0}};
  std::memcpy(dR[0], dw, sizeof(M3));
  std::memcpy(dR[1], dx, sizeof(M3));
  std::memcpy(dR[2], dy, sizeof(M3));
  std::memcpy(dR[3], dz, sizeof(M3));
}

// All intermediate quantities of the projection of one Gaussian.
struct Proj {
  bool kept;
  double p[3];         // camera-space mean
  double zkey;         // float32 camera z that orders and culls (see project_one)
  double qn[4], qnorm; // normalised quaternion and the norm of the input
  M3 Rq;               // rotation of the Gaussian
  double S[3];         // exp(log_scale)
  M3 Sigma;            // world covariance
  M3 V;                // camera covariance R Sigma R^T
  double J[2][3];      // projection Jacobian
  double cov[3];       // 2D covariance (a, b, c) including the low-pass
  double det;
  double conic[3];     // (k1, k2, k3) = (c, -b, a) / det
  double u[2];         // pixel mean
  double o;            // opacity
  double extent;       // sqrt(2 ln(255 o) lambda_max)
  int radius;          // ceil(extent)
};

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

Proj project_one(const Cam& cam, const double mean[3], const double ls[3], const double q[4], double opl) {
  Proj P;
  std::memset(&P, 0, sizeof(P));
  P.kept = false;
  double in[11] = {mean[0], mean[1], mean[2], ls[0], ls[1], ls[2], q[0], q[1], q[2], q[3], opl};
  if (!finite_all(in, 11)) return P;
  for (int i = 0; i < 3; ++i)
    P.p[i] = cam.R[i][0] * mean[0] + cam.R[i][1] * mean[1] + cam.R[i][2] * mean[2] + cam.t[i];
  const double x = P.p[0], y = P.p[1], z = P.p[2];
  // The depth order (a permutation) and the near-plane cull are decisions
  // taken from a float32 camera z in the GPU path; both sides take them on
  // the same float32 value: ((R20 m0 + R21 m1) + R22 m2) + t2, each operation
  // rounded to float32 (inputs are float32, so they convert exactly).
  {
    volatile float a = (float)cam.R[2][0] * (float)mean[0];
    volatile float b = (float)cam.R[2][1] * (float)mean[1];
    volatile float c = (float)cam.R[2][2] * (float)mean[2];
    volatile float ab = a + b;
    volatile float abc = ab + c;
    volatile float zf = abc + (float)cam.t[2];
    P.zkey = (double)zf;
  }
  if (!(P.zkey > (double)(float)cam.znear)) return P;
  P.qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(P.qnorm > 0)) return P;
  for (int i = 0; i < 4; ++i) P.qn[i] = q[i] / P.qnorm;
  quat_to_rot(P.qn[0], P.qn[1], P.qn[2], P.qn[3], P.Rq);
  for (int i = 0; i < 3; ++i) P.S[i] = std::exp(ls[i]);
  // Sigma = Rq diag(S^2) Rq^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += P.Rq[i][k] * P.S[k] * P.S[k] * P.Rq[j][k];
      P.Sigma[i][j] = s;
    }
  M3 Rt;
  transpose3(cam.R, Rt);
  M3 tmp;
  matmul3(cam.R, P.Sigma, tmp);
  matmul3(tmp, Rt, P.V);
  P.J[0][0] = cam.fx / z; P.J[0][1] = 0;           P.J[0][2] = -cam.fx * x / (z * z);
  P.J[1][0] = 0;          P.J[1][1] = cam.fy / z;  P.J[1][2] = -cam.fy * y / (z * z);
  double C2[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) s += P.J[i][k] * P.V[k][l] * P.J[j][l];
      C2[i][j] = s;
    }
  const double a = C2[0][0] + 0.3, b = C2[0][1], c = C2[1][1] + 0.3;
  P.cov[0] = a; P.cov[1] = b; P.cov[2] = c;
  P.det = a * c - b * b;
  if (!(P.det > 0)) return P;
  P.conic[0] = c / P.det;
  P.conic[1] = -b / P.det;
  P.conic[2] = a / P.det;
  P.u[0] = cam.fx * x / z + cam.cx;
  P.u[1] = cam.fy * y / z + cam.cy;
  P.o = 1.0 / (1.0 + std::exp(-opl));
  if (P.o < 1.0 / 255.0) return P;
  const double lmax = 0.5 * (a + c) + std::sqrt(0.25 * (a - c) * (a - c) + b * b);
  P.extent = std::sqrt(2.0 * std::log(255.0 * P.o) * lmax);
  P.radius = (int)std::ceil(P.extent);
  P.kept = true;
  return P;
}

// Kept Gaussians in ascending (depth key, id) order. The key is the float32
// camera z of the projection (`zkey`) or, for measuring what that choice
// changes, the float64 camera z (`depth`).
std::vector<int64_t> depth_order(int64_t n, const double* zkey, const uint8_t* kept) {
  std::vector<int64_t> ord;
  ord.reserve(n);
  for (int64_t k = 0; k < n; ++k)
    if (kept[k]) ord.push_back(k);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return zkey[a] < zkey[b]; });
  return ord;
}

struct Step {
  int64_t k;
  double alpha, T, G;  // alpha used, transmittance before, exp(p)
  bool clamped;
  double dx, dy;
};

// Front-to-back compositing of one pixel. Records the contributing steps when
// `steps` is non-null and returns the margin to the nearest discontinuity.
// With `gap_margin` set, the margin also takes the relative depth gap between
// consecutive Gaussians that take part in the pixel (those added, and the one
// that stops it): where two of them are nearly level, an order decided in
// another precision may swap them.
double composite_pixel(int i, int j, const std::vector<int64_t>& ord, const double* mean2d, int64_t n,
                       const double* conic, const double* depth, const double* opacity, const double* color,
                       const double* mp, double out[6], std::vector<Step>* steps, int* ncontrib,
                       bool gap_margin = false) {
  double T = 1.0, C[3] = {0, 0, 0}, D = 0, M = 0;
  double margin = 1e30;
  double zprev = -1.0;
  int nc = 0;
  for (size_t s = 0; s < ord.size(); ++s) {
    const int64_t k = ord[s];
    const double dx = mean2d[k] - i, dy = mean2d[n + k] - j;
    const double k1 = conic[k], k2 = conic[n + k], k3 = conic[2 * n + k];
    const double p = -0.5 * (k1 * dx * dx + k3 * dy * dy) - k2 * dx * dy;
    if (p > 0) continue;
    const double G = std::exp(p);
    const double araw = opacity[k] * G;
    const double alpha = std::min(0.99, araw);
    if (araw > 0.99 / 1.01 && araw < 0.99 * 1.01) margin = std::min(margin, std::fabs(araw - 0.99));
    if (araw > (1.0 / 255.0) / 1.01 && araw < (1.0 / 255.0) * 1.01)
      margin = std::min(margin, std::fabs(std::log(255.0 * araw)));
    if (alpha < 1.0 / 255.0) continue;
    const double Tn = T * (1.0 - alpha);
    margin = std::min(margin, std::fabs(std::log(Tn / 1e-4)));
    if (gap_margin) {
      if (zprev > 0) margin = std::min(margin, std::fabs(depth[k] - zprev) / depth[k]);
      zprev = depth[k];
    }
    if (Tn < 1e-4) break;
    if (steps) steps->push_back(Step{k, alpha, T, G, araw > 0.99, dx, dy});
    for (int c = 0; c < 3; ++c) C[c] += alpha * T * color[c * n + k];
    D += alpha * T * depth[k];
    M += alpha * T * mp[k];
    T = Tn;
    ++nc;
  }
  out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = D; out[4] = M; out[5] = T;
  if (ncontrib) *ncontrib = nc;
  return margin;
}

}  // namespace

extern "C" {

int or_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Projection of n Gaussians (planar inputs: mean[3n], log_scale[3n], quat[4n], opl[n]).
// Outputs are planar; culled Gaussians have kept = 0 and undefined values.
int or_project(int64_t n, const double* mean, const double* log_scale, const double* quat, const double* opl,
               const double* camv, double* mean2d, double* conic, double* cov2d, double* depth,
               double* opacity, double* extent, int32_t* radius, uint8_t* kept, double* zkey) {
  const Cam cam = read_cam(camv);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    const double m[3] = {mean[k], mean[n + k], mean[2 * n + k]};
    const double l[3] = {log_scale[k], log_scale[n + k], log_scale[2 * n + k]};
    const double q[4] = {quat[k], quat[n + k], quat[2 * n + k], quat[3 * n + k]};
    const Proj P = project_one(cam, m, l, q, opl[k]);
    kept[k] = P.kept ? 1 : 0;
    mean2d[k] = P.u[0]; mean2d[n + k] = P.u[1];
    for (int c = 0; c < 3; ++c) {
      conic[c * n + k] = P.conic[c];
      cov2d[c * n + k] = P.cov[c];
    }
    depth[k] = P.p[2];
    zkey[k] = P.zkey;
    opacity[k] = P.o;
    extent[k] = P.extent;
    radius[k] = P.radius;
  }
  return 0;
}

// Tile-free render. If npix >= 0, only the listed pixel indices (y*W + x) are
// rendered and outputs are indexed by position in that list; otherwise all W*H.
// order_f64 = 1 orders by the float64 camera z instead of the float32 key
// and adds the depth-gap term to the margin (a measurement aid; the parity
// reference is order_f64 = 0).
int or_render(int64_t n, const double* mean2d, const double* conic, const double* depth, const double* zkey,
              const double* opacity, const double* color, const double* mp, const uint8_t* kept, int W, int H,
              const double* bg,
              int64_t npix, const int64_t* pix, double* C, double* D, double* M, double* T, double* margin,
              int32_t* ncontrib, int order_f64) {
  const std::vector<int64_t> ord = depth_order(n, order_f64 ? depth : zkey, kept);
  const int64_t P = npix >= 0 ? npix : (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < P; ++q) {
    const int64_t id = npix >= 0 ? pix[q] : q;
    const int i = (int)(id % W), j = (int)(id / W);
    double out[6];
    int nc = 0;
    const double mg =
        composite_pixel(i, j, ord, mean2d, n, conic, depth, opacity, color, mp, out, nullptr, &nc, order_f64 != 0);
    for (int c = 0; c < 3; ++c) C[c * P + q] = out[c] + out[5] * bg[c];
    D[q] = out[3];
    M[q] = out[4];
    T[q] = out[5];
    margin[q] = mg;
    ncontrib[q] = nc;
  }
  return 0;
}

// Reverse mode through the render. Upstream per-pixel adjoints gC[3P], gD[P],
// gM[P], gT[P] (gT is the adjoint of the final transmittance; the background
// term of C is added here). Output per-Gaussian 2D adjoints, planar [10][n]:
// (u_x, u_y, k1, k2, k3, opacity, c_r, c_g, c_b, depth).
int or_render_backward(int64_t n, const double* mean2d, const double* conic, const double* depth,
                       const double* zkey, const double* opacity, const double* color, const double* mp,
                       const uint8_t* kept, int W,
                       int H, const double* bg, int64_t npix, const int64_t* pix, const double* gC,
                       const double* gD, const double* gM, const double* gT, double* g2d) {
  const std::vector<int64_t> ord = depth_order(n, zkey, kept);
  const int64_t P = npix >= 0 ? npix : (int64_t)W * H;
  std::memset(g2d, 0, sizeof(double) * 10 * n);
#pragma omp parallel
  {
    std::vector<double> acc(10 * (size_t)n, 0.0);
    std::vector<Step> steps;
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < P; ++q) {
      const int64_t id = npix >= 0 ? pix[q] : q;
      const int i = (int)(id % W), j = (int)(id / W);
      steps.clear();
      double out[6];
      composite_pixel(i, j, ord, mean2d, n, conic, depth, opacity, color, mp, out, &steps, nullptr);
      const double gc[3] = {gC[q], gC[P + q], gC[2 * P + q]};
      const double gd = gD[q], gm = gM ? gM[q] : 0.0;
      // adjoint of the transmittance after the last step: final T output and
      // the background term C += T_final * bg
      double Tbar = (gT ? gT[q] : 0.0) + gc[0] * bg[0] + gc[1] * bg[1] + gc[2] * bg[2];
      for (int s = (int)steps.size() - 1; s >= 0; --s) {
        const Step& st = steps[s];
        const int64_t k = st.k;
        const double ck[3] = {color[k], color[n + k], color[2 * n + k]};
        const double v = gc[0] * ck[0] + gc[1] * ck[1] + gc[2] * ck[2] + gd * depth[k] + gm * mp[k];
        // forward step: X += alpha T x ; T_next = T (1 - alpha)
        const double abar = st.T * v - Tbar * st.T;
        const double w = st.alpha * st.T;
        for (int c = 0; c < 3; ++c) acc[(6 + c) * n + k] += w * gc[c];
        acc[9 * n + k] += w * gd;
        Tbar = v * st.alpha + Tbar * (1.0 - st.alpha);
        if (st.clamped) continue;  // alpha = 0.99 does not depend on o or p
        const double obar = abar * st.G;
        const double pbar = abar * st.alpha;
        const double k1 = conic[k], k2 = conic[n + k], k3 = conic[2 * n + k];
        const double dx = st.dx, dy = st.dy;
        acc[0 * n + k] += pbar * (-k1 * dx - k2 * dy);
        acc[1 * n + k] += pbar * (-k3 * dy - k2 * dx);
        acc[2 * n + k] += pbar * (-0.5 * dx * dx);
        acc[3 * n + k] += pbar * (-dx * dy);
        acc[4 * n + k] += pbar * (-0.5 * dy * dy);
        acc[5 * n + k] += obar;
      }
    }
#pragma omp critical
    for (size_t e = 0; e < acc.size(); ++e) g2d[e] += acc[e];
  }
  return 0;
}

// Chain the 2D adjoints through the projection. Outputs (planar, overwritten):
// dmean[3n], dlog_scale[3n], dquat[4n], dopl[n], dcolor[3n], and the pose
// twist adjoint dpose[6] = (rho, phi) for T <- Exp(xi) T.
int or_project_backward(int64_t n, const double* mean, const double* log_scale, const double* quat,
                        const double* opl, const double* camv, const double* g2d, double* dmean,
                        double* dlog_scale, double* dquat, double* dopl, double* dcolor, double* dpose) {
  const Cam cam = read_cam(camv);
  double pose_acc[6] = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
  {
    double pl[6] = {0, 0, 0, 0, 0, 0};
#pragma omp for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
      const double m[3] = {mean[k], mean[n + k], mean[2 * n + k]};
      const double l[3] = {log_scale[k], log_scale[n + k], log_scale[2 * n + k]};
      const double q[4] = {quat[k], quat[n + k], quat[2 * n + k], quat[3 * n + k]};
      for (int c = 0; c < 3; ++c) {
        dmean[c * n + k] = 0;
        dlog_scale[c * n + k] = 0;
        dcolor[c * n + k] = g2d[(6 + c) * n + k];
      }
      for (int c = 0; c < 4; ++c) dquat[c * n + k] = 0;
      dopl[k] = 0;
      const Proj P = project_one(cam, m, l, q, opl[k]);
      if (!P.kept) continue;
      const double ub[2] = {g2d[k], g2d[n + k]};
      const double kb[3] = {g2d[2 * n + k], g2d[3 * n + k], g2d[4 * n + k]};
      const double ob = g2d[5 * n + k], zb = g2d[9 * n + k];
      const double x = P.p[0], y = P.p[1], z = P.p[2];
      // conic -> 2D covariance: covbar = -Q G Q with Q the conic matrix and G
      // the symmetric adjoint of Q (off-diagonal halves)
      const double Q[2][2] = {{P.conic[0], P.conic[1]}, {P.conic[1], P.conic[2]}};
      const double Gm[2][2] = {{kb[0], 0.5 * kb[1]}, {0.5 * kb[1], kb[2]}};
      double QG[2][2], cb[2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) QG[i][j] = Q[i][0] * Gm[0][j] + Q[i][1] * Gm[1][j];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) cb[i][j] = -(QG[i][0] * Q[0][j] + QG[i][1] * Q[1][j]);
      // cov2d = J V J^T + 0.3 I  ->  Vbar = J^T cb J ; Jbar = 2 cb J V
      M3 Vb;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) s += P.J[i][a] * cb[i][j] * P.J[j][b];
          Vb[a][b] = s;
        }
      double Jb[2][3];
      for (int i = 0; i < 2; ++i)
        for (int a = 0; a < 3; ++a) {
          double s = 0;
          for (int j = 0; j < 2; ++j)
            for (int b = 0; b < 3; ++b) s += cb[i][j] * P.J[j][b] * P.V[b][a];
          Jb[i][a] = 2.0 * s;
        }
      double pb[3] = {0, 0, 0};
      const double fx = cam.fx, fy = cam.fy;
      pb[0] += Jb[0][2] * (-fx / (z * z));
      pb[1] += Jb[1][2] * (-fy / (z * z));
      pb[2] += Jb[0][0] * (-fx / (z * z)) + Jb[0][2] * (2 * fx * x / (z * z * z)) + Jb[1][1] * (-fy / (z * z)) +
               Jb[1][2] * (2 * fy * y / (z * z * z));
      // pixel mean
      pb[0] += ub[0] * fx / z;
      pb[2] += ub[0] * (-fx * x / (z * z));
      pb[1] += ub[1] * fy / z;
      pb[2] += ub[1] * (-fy * y / (z * z));
      // composited depth is the camera z of the mean
      pb[2] += zb;
      // pose twist: p' = Exp(xi) p -> rho += pb, phi += p x pb
      pl[0] += pb[0]; pl[1] += pb[1]; pl[2] += pb[2];
      pl[3] += y * pb[2] - z * pb[1];
      pl[4] += z * pb[0] - x * pb[2];
      pl[5] += x * pb[1] - y * pb[0];
      // pose twist through V = R Sigma R^T: phi += -2 a with [a]_x = V Vb - Vb V
      M3 A1, A2;
      matmul3(P.V, Vb, A1);
      matmul3(Vb, P.V, A2);
      pl[3] += -2.0 * (A1[2][1] - A2[2][1]);
      pl[4] += -2.0 * (A1[0][2] - A2[0][2]);
      pl[5] += -2.0 * (A1[1][0] - A2[1][0]);
      // mean: p = R mu + t
      for (int c = 0; c < 3; ++c)
        dmean[c * n + k] = cam.R[0][c] * pb[0] + cam.R[1][c] * pb[1] + cam.R[2][c] * pb[2];
      // Sigma = R^T Vb R (world)
      M3 Rt, tmp, Sb;
      transpose3(cam.R, Rt);
      matmul3(Rt, Vb, tmp);
      matmul3(tmp, cam.R, Sb);
      // Sigma = M M^T, M = Rq diag(S): Mbar = 2 Sb M
      M3 Mm, Mb;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mm[i][j] = P.Rq[i][j] * P.S[j];
      matmul3(Sb, Mm, Mb);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mb[i][j] *= 2.0;
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int i = 0; i < 3; ++i) s += P.Rq[i][c] * Mb[i][c];
        dlog_scale[c * n + k] = s * P.S[c];
      }
      M3 Rb;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Rb[i][j] = Mb[i][j] * P.S[j];
      M3 dR[4];
      quat_rot_derivs(P.qn[0], P.qn[1], P.qn[2], P.qn[3], dR);
      double qnb[4];
      for (int c = 0; c < 4; ++c) {
        double s = 0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) s += Rb[i][j] * dR[c][i][j];
        qnb[c] = s;
      }
      const double dotq = qnb[0] * P.qn[0] + qnb[1] * P.qn[1] + qnb[2] * P.qn[2] + qnb[3] * P.qn[3];
      for (int c = 0; c < 4; ++c) dquat[c * n + k] = (qnb[c] - P.qn[c] * dotq) / P.qnorm;
      dopl[k] = ob * P.o * (1.0 - P.o);
    }
#pragma omp critical
    for (int c = 0; c < 6; ++c) pose_acc[c] += pl[c];
  }
  for (int c = 0; c < 6; ++c) dpose[c] = pose_acc[c];
  return 0;
}

}  // extern "C"
