// Bone transforms from the body pose (Sec. 4.2, Eq. 8), host, double
// precision; their adjoint; and the pose refiner of Sec. 4.1 (Eq. 5-6).
//
// The observed pose theta^o gives each joint a rotation: R(w_j), or
// R(delta_j) R(w_j) when the pose refiner's adjustment delta is present
// (Eq. 6 composes the adjustment with the estimated angle).  World
// transforms compose down the tree: A_root = [R_root | J_root],
// A_j = A_parent o [R_j | J_j - J_parent].  The skinning transform of bone
// j carries a canonical (rest-pose) point to the observation:
// B_j = A_j o [I | -J_j].  The warp of Eq. 7-8 needs the inverse,
// G_j = B_j^-1 = [R^T | -R^T t], which maps observed points to canonical
// ones.  Rotations use Rodrigues' formula.
//
// The adjoint differentiates this same code with forward-mode dual numbers
// (one pass per input angle): exact derivatives, and cheap for 24 joints.
#include <cmath>
#include <cstring>

#include "host_common.h"

namespace mnr {

struct Dual {  // value + derivative along one seeded input
  double v, d;
  Dual(double v_ = 0.0, double d_ = 0.0) : v(v_), d(d_) {}
};
static inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
static inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
static inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
static inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
static inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
static inline Dual sqrt(Dual a) {
  const double r = std::sqrt(a.v);
  return {r, a.d / (2.0 * r)};
}
static inline Dual sin(Dual a) { return {std::sin(a.v), a.d * std::cos(a.v)}; }
static inline Dual cos(Dual a) { return {std::cos(a.v), -a.d * std::sin(a.v)}; }
static inline double value(double a) { return a; }
static inline double value(Dual a) { return a.v; }
using std::cos;
using std::sin;
using std::sqrt;

template <typename T>
static void rodrigues(const T w[3], T R[9]) {
  const T th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + T(0.0));
  T K[9] = {T(0.0), -w[2], w[1], w[2], T(0.0), -w[0], -w[1], w[0], T(0.0)};
  T s, c1;
  if (value(th) < 1e-12) {  // first-order expansion: R = I + [w]x (exact derivative at w = 0)
    s = T(1.0);
    c1 = T(0.0);
  } else {
    for (T& k : K) k = k / th;
    s = sin(th);
    c1 = T(1.0) - cos(th);
  }
  T K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T acc = T(0.0);
      for (int k = 0; k < 3; ++k) acc = acc + K[i * 3 + k] * K[k * 3 + j];
      K2[i * 3 + j] = acc;
    }
  for (int i = 0; i < 9; ++i) R[i] = T(i % 4 == 0 ? 1.0 : 0.0) + s * K[i] + c1 * K2[i];
}

template <typename T>
static void matmul3(const T* A, const T* B, T* C) {
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      T acc = T(0.0);
      for (int m = 0; m < 3; ++m) acc = acc + A[i * 3 + m] * B[m * 3 + k];
      C[i * 3 + k] = acc;
    }
}

// G [n][12] from joint angles w [3n] and optional adjustments dl [3n].
template <typename T>
static void fk_t(const mnr_pose* pose, const T* w, const T* dl, T* G) {
  const int n = pose->n_joints;
  T Ar[MNR_MAX_BONES][9], At[MNR_MAX_BONES][3];
  for (int j = 0; j < n; ++j) {
    T R[9];
    rodrigues(w + 3 * j, R);
    if (dl) {
      T D[9], RD[9];
      rodrigues(dl + 3 * j, D);
      matmul3(D, R, RD);
      std::memcpy((void*)R, (const void*)RD, sizeof(R));
    }
    const float* Jj = pose->rest_joints + 3 * j;
    const int p = pose->parent[j];
    if (p < 0) {
      std::memcpy((void*)Ar[j], (const void*)R, sizeof(R));
      for (int a = 0; a < 3; ++a) At[j][a] = T((double)Jj[a]);
    } else {
      const float* Jp = pose->rest_joints + 3 * p;
      const double off[3] = {(double)Jj[0] - Jp[0], (double)Jj[1] - Jp[1], (double)Jj[2] - Jp[2]};
      matmul3(Ar[p], R, Ar[j]);
      for (int i = 0; i < 3; ++i)
        At[j][i] = Ar[p][i * 3 + 0] * T(off[0]) + Ar[p][i * 3 + 1] * T(off[1]) + Ar[p][i * 3 + 2] * T(off[2]) +
                   At[p][i];
    }
  }
  for (int j = 0; j < n; ++j) {
    const float* Jj = pose->rest_joints + 3 * j;
    T bt[3];  // translation of B_j = A_j o [I | -J_j]
    for (int i = 0; i < 3; ++i)
      bt[i] = At[j][i] - (Ar[j][i * 3 + 0] * T((double)Jj[0]) + Ar[j][i * 3 + 1] * T((double)Jj[1]) +
                          Ar[j][i * 3 + 2] * T((double)Jj[2]));
    T* g = G + 12 * j;
    for (int i = 0; i < 3; ++i) {
      for (int k = 0; k < 3; ++k) g[i * 4 + k] = Ar[j][k * 3 + i];  // R^T
      g[i * 4 + 3] = -(Ar[j][0 * 3 + i] * bt[0] + Ar[j][1 * 3 + i] * bt[1] + Ar[j][2 * 3 + i] * bt[2]);
    }
  }
}

mnr_status validate_pose(const mnr_pose* pose) {
  if (!pose || !pose->parent || !pose->rest_joints || !pose->axis_angle) return fail(MNR_E_INVALID, "pose: null pointer");
  const int n = pose->n_joints;
  if (n < 1 || n > MNR_MAX_BONES) return fail(MNR_E_SHAPE, "pose: n_joints must be in [1, %d], got %d", MNR_MAX_BONES, n);
  if (pose->parent[0] != -1) return fail(MNR_E_INVALID, "pose: joint 0 must be the root (parent -1)");
  for (int j = 1; j < n; ++j)
    if (pose->parent[j] < 0 || pose->parent[j] >= j)
      return fail(MNR_E_INVALID, "pose: parent[%d] = %d must precede the joint", j, pose->parent[j]);
  for (int i = 0; i < 3 * n; ++i)
    if (!std::isfinite(pose->axis_angle[i]) || !std::isfinite(pose->rest_joints[i]) ||
        (pose->delta && !std::isfinite(pose->delta[i])))
      return fail(MNR_E_INVALID, "pose: non-finite joint angle, adjustment or rest joint");
  return MNR_OK;
}

void fk_bones_f64(const mnr_pose* pose, double* G /* [n][12] */) {
  const int n = pose->n_joints;
  double w[3 * MNR_MAX_BONES], dl[3 * MNR_MAX_BONES];
  for (int i = 0; i < 3 * n; ++i) {
    w[i] = pose->axis_angle[i];
    dl[i] = pose->delta ? pose->delta[i] : 0.0;
  }
  fk_t<double>(pose, w, pose->delta ? dl : nullptr, G);
}

// Axis-angle of a rotation (principal branch: angle theta in [0, pi]).
// With R = cos(theta) I + sin(theta) [a]x + (1 - cos(theta)) a a^T, the
// skew part gives v = sin(theta) a and the trace cos(theta); theta =
// atan2(|v|, cos(theta)).  Near theta = pi, where v vanishes, the axis
// comes from the symmetric part, a a^T = (S - cos(theta) I) /
// (1 - cos(theta)), its sign from v.
static void rotation_log(const double R[9], double w[3]) {
  const double v[3] = {0.5 * (R[7] - R[5]), 0.5 * (R[2] - R[6]), 0.5 * (R[3] - R[1])};
  const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  const double s = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double th = std::atan2(s, c);
  if (th < 1e-6) {  // theta / sin(theta) = 1 + theta^2 / 6 + O(theta^4)
    for (int i = 0; i < 3; ++i) w[i] = v[i] * (1.0 + th * th / 6.0);
    return;
  }
  if (c > -0.9) {
    for (int i = 0; i < 3; ++i) w[i] = v[i] * (th / s);
    return;
  }
  double M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = (0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? c : 0.0)) / (1.0 - c);
  int k = 0;
  for (int i = 1; i < 3; ++i)
    if (M[4 * i] > M[4 * k]) k = i;
  const double ak = std::sqrt(M[4 * k]);
  double a[3];
  for (int j = 0; j < 3; ++j) a[j] = M[3 * k + j] / ak;
  const double dot = a[0] * v[0] + a[1] * v[1] + a[2] * v[2];
  const double sg = dot < 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i) w[i] = sg * th * a[i];
}

void pose_angles_f64(const mnr_pose* pose, double* omega) {
  const int n = pose->n_joints;
  for (int j = 0; j < n; ++j) {
    double w[3] = {pose->axis_angle[3 * j], pose->axis_angle[3 * j + 1], pose->axis_angle[3 * j + 2]};
    if (!pose->delta) {
      for (int i = 0; i < 3; ++i) omega[3 * j + i] = w[i];
      continue;
    }
    const double d[3] = {pose->delta[3 * j], pose->delta[3 * j + 1], pose->delta[3 * j + 2]};
    double Rw[9], Rd[9], R[9];
    rodrigues<double>(w, Rw);
    rodrigues<double>(d, Rd);
    matmul3<double>(Rd, Rw, R);
    rotation_log(R, omega + 3 * j);
  }
}

// Refiner layers in double precision; hidden activations kept for the adjoint.
static constexpr int MAX_REFINER_WIDTH = 1024;

static mnr_status validate_refiner(const mnr_refiner* r, int n) {
  if (!r) return fail(MNR_E_INVALID, "refiner: null pointer");
  if (r->n_layers < 1 || r->n_layers > MNR_MAX_LAYERS)
    return fail(MNR_E_SHAPE, "refiner: n_layers must be in [1, %d]", MNR_MAX_LAYERS);
  if (n < 1 || n > MNR_MAX_BONES) return fail(MNR_E_SHAPE, "refiner: bad joint count %d", n);
  if (r->width[0] != 3 * n || r->width[r->n_layers] != 3 * n)
    return fail(MNR_E_SHAPE, "refiner: input and output widths must be 3 n_joints = %d", 3 * n);
  for (int k = 0; k <= r->n_layers; ++k)
    if (r->width[k] < 1 || r->width[k] > MAX_REFINER_WIDTH) return fail(MNR_E_SHAPE, "refiner: width out of range");
  for (int k = 0; k < r->n_layers; ++k)
    if (!r->w[k]) return fail(MNR_E_INVALID, "refiner: null weight %d", k);
  return MNR_OK;
}

// act[k] = input of layer k (act[0] = omega, act[k] = ReLU(W_{k-1} act[k-1]));
// out = W_last act[last].
static void refiner_forward(const mnr_refiner* r, const float* omega, double act[][MAX_REFINER_WIDTH], double* out) {
  for (int i = 0; i < r->width[0]; ++i) act[0][i] = omega[i];
  for (int k = 0; k < r->n_layers; ++k) {
    const int K = r->width[k], M = r->width[k + 1];
    double* dst = (k + 1 < r->n_layers) ? act[k + 1] : out;
    for (int m = 0; m < M; ++m) {
      double acc = 0.0;
      for (int i = 0; i < K; ++i) acc += (double)r->w[k][(size_t)m * K + i] * act[k][i];
      dst[m] = (k + 1 < r->n_layers) ? (acc > 0.0 ? acc : 0.0) : acc;
    }
  }
}

}  // namespace mnr

using namespace mnr;

extern "C" mnr_status mnr_fk_bones(const mnr_pose* pose, float* G_out) {
  clear_error();
  if (mnr_status s = validate_pose(pose)) return s;
  if (!G_out) return fail(MNR_E_INVALID, "fk: null output");
  double G[MNR_MAX_BONES * 12];
  fk_bones_f64(pose, G);
  for (int i = 0; i < 12 * pose->n_joints; ++i) G_out[i] = (float)G[i];
  return MNR_OK;
}

extern "C" mnr_status mnr_fk_backward(const mnr_pose* pose, const float* grad_G, float* grad_delta,
                                      float* grad_axis_angle) {
  clear_error();
  if (mnr_status s = validate_pose(pose)) return s;
  if (!grad_G) return fail(MNR_E_INVALID, "fk_backward: null grad_G");
  const int n = pose->n_joints;
  Dual w[3 * MNR_MAX_BONES], dl[3 * MNR_MAX_BONES], G[12 * MNR_MAX_BONES];
  for (int i = 0; i < 3 * n; ++i) {
    w[i] = Dual(pose->axis_angle[i]);
    dl[i] = Dual(pose->delta ? pose->delta[i] : 0.0);
  }
  // With no refiner adjustment the composition is skipped (R(0) = I); the
  // derivative with respect to delta is then taken at delta = 0.
  for (int which = 0; which < 2; ++which) {
    float* out = which == 0 ? grad_delta : grad_axis_angle;
    if (!out) continue;
    Dual* x = which == 0 ? dl : w;
    for (int i = 0; i < 3 * n; ++i) {
      x[i].d = 1.0;
      fk_t<Dual>(pose, w, dl, G);
      x[i].d = 0.0;
      double acc = 0.0;
      for (int k = 0; k < 12 * n; ++k) acc += (double)grad_G[k] * G[k].d;
      out[i] = (float)acc;
    }
  }
  return MNR_OK;
}

extern "C" mnr_status mnr_refiner_apply(const mnr_refiner* r, int32_t n_joints, const float* omega, float* delta) {
  clear_error();
  if (mnr_status s = validate_refiner(r, n_joints)) return s;
  if (!omega || !delta) return fail(MNR_E_INVALID, "refiner: null pointer");
  static thread_local double act[MNR_MAX_LAYERS][MAX_REFINER_WIDTH];
  double out[3 * MNR_MAX_BONES];
  refiner_forward(r, omega, act, out);
  for (int i = 0; i < 3 * n_joints; ++i) delta[i] = (float)out[i];
  return MNR_OK;
}

extern "C" mnr_status mnr_refiner_backward(const mnr_refiner* r, int32_t n_joints, const float* omega,
                                           const float* grad_delta, float* const* grad_w) {
  clear_error();
  if (mnr_status s = validate_refiner(r, n_joints)) return s;
  if (!omega || !grad_delta || !grad_w) return fail(MNR_E_INVALID, "refiner_backward: null pointer");
  for (int k = 0; k < r->n_layers; ++k)
    if (!grad_w[k]) return fail(MNR_E_INVALID, "refiner_backward: null gradient %d", k);
  static thread_local double act[MNR_MAX_LAYERS][MAX_REFINER_WIDTH];
  static thread_local double g[MAX_REFINER_WIDTH], gp[MAX_REFINER_WIDTH];
  double out[3 * MNR_MAX_BONES];
  refiner_forward(r, omega, act, out);
  for (int i = 0; i < 3 * n_joints; ++i) g[i] = grad_delta[i];  // dL/d(output of the last layer)
  for (int k = r->n_layers - 1; k >= 0; --k) {
    const int K = r->width[k], M = r->width[k + 1];
    for (int m = 0; m < M; ++m)
      for (int i = 0; i < K; ++i) grad_w[k][(size_t)m * K + i] += (float)(g[m] * act[k][i]);
    if (k == 0) break;
    for (int i = 0; i < K; ++i) {
      double acc = 0.0;
      for (int m = 0; m < M; ++m) acc += (double)r->w[k][(size_t)m * K + i] * g[m];
      gp[i] = act[k][i] > 0.0 ? acc : 0.0;  // through the ReLU that produced act[k]
    }
    for (int i = 0; i < K; ++i) g[i] = gp[i];
  }
  return MNR_OK;
}

extern "C" mnr_status mnr_refiner_adam(const mnr_refiner* r, int32_t n_joints, float* const* w, float* const* grad_w,
                                       float* const* m, float* const* v, int32_t step, float lr, float beta1,
                                       float beta2, float eps) {
  clear_error();
  if (mnr_status s = validate_refiner(r, n_joints)) return s;
  if (!w || !grad_w || !m || !v) return fail(MNR_E_INVALID, "refiner_adam: null pointer");
  if (step < 1) return fail(MNR_E_INVALID, "refiner_adam: step must be >= 1");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(MNR_E_INVALID, "refiner_adam: bad hyper-parameters");
  for (int k = 0; k < r->n_layers; ++k)
    if (!w[k] || !grad_w[k] || !m[k] || !v[k]) return fail(MNR_E_INVALID, "refiner_adam: null layer %d", k);
  const double bc1 = 1.0 - std::pow((double)beta1, (double)step);
  const double bc2 = 1.0 - std::pow((double)beta2, (double)step);
  for (int k = 0; k < r->n_layers; ++k) {
    const size_t n = (size_t)r->width[k] * r->width[k + 1];
    for (size_t i = 0; i < n; ++i) {
      const double g = grad_w[k][i];
      const double mi = beta1 * (double)m[k][i] + (1.0 - beta1) * g;
      const double vi = beta2 * (double)v[k][i] + (1.0 - beta2) * g * g;
      m[k][i] = (float)mi;
      v[k][i] = (float)vi;
      w[k][i] = (float)((double)w[k][i] - lr * (mi / bc1) / (std::sqrt(vi / bc2) + eps));
      grad_w[k][i] = 0.f;
    }
  }
  return MNR_OK;
}
