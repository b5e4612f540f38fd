// Bone transforms from the body pose (Sec. 4.2, Eq. 8), host, double precision.
//
// The observed pose theta^o gives each joint a rotation (axis-angle).  World
// transforms compose down the tree: A_root = [R(w_root) | J_root],
// A_j = A_parent o [R(w_j) | J_j - J_parent].  The skinning transform of
// bone j carries a canonical (rest-pose) point to the observation:
// B_j = A_j o [I | -J_j].  The warp of Eq. 7-8 needs the inverse,
// G_j = B_j^-1 = [R^T | -R^T t], which maps observed points to canonical
// ones.  Rotations use Rodrigues' formula.
#include <cmath>
#include <cstring>

#include "host_common.h"

namespace mnr {

static void rodrigues(const double w[3], double R[9]) {
  const double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  double s, c1;
  if (th < 1e-12) {  // first-order expansion: R = I + [w]x
    s = 1.0;
    c1 = 0.0;
  } else {
    for (double& k : K) k /= th;
    s = std::sin(th);
    c1 = 1.0 - std::cos(th);
  }
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += K[i * 3 + k] * K[k * 3 + j];
      K2[i * 3 + j] = acc;
    }
  for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + s * K[i] + c1 * K2[i];
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
    if (!std::isfinite(pose->axis_angle[i]) || !std::isfinite(pose->rest_joints[i]))
      return fail(MNR_E_INVALID, "pose: non-finite joint angle or rest joint");
  return MNR_OK;
}

void fk_bones_f64(const mnr_pose* pose, double* G /* [n][12] */) {
  const int n = pose->n_joints;
  double Ar[MNR_MAX_BONES][9], At[MNR_MAX_BONES][3];
  for (int j = 0; j < n; ++j) {
    double w[3] = {pose->axis_angle[3 * j], pose->axis_angle[3 * j + 1], pose->axis_angle[3 * j + 2]};
    double R[9];
    rodrigues(w, R);
    const float* Jj = pose->rest_joints + 3 * j;
    const int p = pose->parent[j];
    if (p < 0) {
      std::memcpy(Ar[j], R, sizeof(R));
      for (int a = 0; a < 3; ++a) At[j][a] = Jj[a];
    } else {
      const float* Jp = pose->rest_joints + 3 * p;
      const double off[3] = {(double)Jj[0] - Jp[0], (double)Jj[1] - Jp[1], (double)Jj[2] - Jp[2]};
      for (int i = 0; i < 3; ++i) {
        for (int k = 0; k < 3; ++k) {
          double acc = 0;
          for (int m = 0; m < 3; ++m) acc += Ar[p][i * 3 + m] * R[m * 3 + k];
          Ar[j][i * 3 + k] = acc;
        }
        At[j][i] = Ar[p][i * 3 + 0] * off[0] + Ar[p][i * 3 + 1] * off[1] + Ar[p][i * 3 + 2] * off[2] + At[p][i];
      }
    }
  }
  for (int j = 0; j < n; ++j) {
    const float* Jj = pose->rest_joints + 3 * j;
    double bt[3];  // translation of B_j = A_j o [I | -J_j]
    for (int i = 0; i < 3; ++i)
      bt[i] = At[j][i] - (Ar[j][i * 3 + 0] * Jj[0] + Ar[j][i * 3 + 1] * Jj[1] + Ar[j][i * 3 + 2] * Jj[2]);
    double* g = G + 12 * j;
    for (int i = 0; i < 3; ++i) {
      for (int k = 0; k < 3; ++k) g[i * 4 + k] = Ar[j][k * 3 + i];  // R^T
      g[i * 4 + 3] = -(Ar[j][0 * 3 + i] * bt[0] + Ar[j][1 * 3 + i] * bt[1] + Ar[j][2 * 3 + i] * bt[2]);
    }
  }
}

}  // namespace mnr

extern "C" mnr_status mnr_fk_bones(const mnr_pose* pose, float* G_out) {
  using namespace mnr;
  clear_error();
  if (mnr_status s = validate_pose(pose)) return s;
  if (!G_out) return fail(MNR_E_INVALID, "fk: null output");
  double G[MNR_MAX_BONES * 12];
  fk_bones_f64(pose, G);
  for (int i = 0; i < 12 * pose->n_joints; ++i) G_out[i] = (float)G[i];
  return MNR_OK;
}
