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

}  // namespace mnr
