// Host-side helpers: thread-local error text, validation, argument packing.
#pragma once
#include <cstdarg>
#include <cstdio>

#include "../../include/metanerf.h"

namespace mnr {

void clear_error();
mnr_status fail(mnr_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
mnr_status validate_pose(const mnr_pose* pose);
void fk_bones_f64(const mnr_pose* pose, double* G);
// Joint angles of the observed pose [3n]: axis_angle, or with the refiner's
// adjustment the axis-angle of R(delta_j) R(axis_angle_j) (angle <= pi).
void pose_angles_f64(const mnr_pose* pose, double* omega);

struct RenderArgs;
struct FieldArgs;
void field_args(FieldArgs& F, const mnr_field* f);
mnr_status validate_field(const mnr_field* f);
mnr_status validate_common(const mnr_field* f, const mnr_motion* m, const mnr_pose* p, const mnr_camera* c, int H,
                           int W, int spp, const mnr_opts* o, const int32_t* pixel_ids, int n_rays, const void* out);
void pack_args(RenderArgs& a, const mnr_field* f, const mnr_motion* m, const mnr_pose* p, const mnr_camera* c, int H,
               int W, int spp, const mnr_opts* o, const int32_t* pixel_ids, int n_rays);
int slot_count(int H, int W, const int32_t* pixel_ids, int n_rays);

}  // namespace mnr
