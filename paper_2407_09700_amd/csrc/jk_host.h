// Host helpers shared by the translation units of the C ABI.
#pragma once

namespace jk {
// Cartesian -> real-solid-harmonic matrix of momentum l ((2l+1) x (l+1)(l+2)/2, row-major).
void solid_harmonics_host(int l, double *T);
// Records a thread-local error message for jk_last_error() and returns code.
int set_error(int code, const char *fmt, ...);
}  // namespace jk
