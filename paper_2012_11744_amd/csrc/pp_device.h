// pp_device.h -- device-side types shared by the HIP sources of the
// pressure-projection library.  Not part of the ABI.
#pragma once

#include "pp_internal.h"

namespace pp {

template <typename T>
struct Acc {
    using type = float;   // FP32 arithmetic for FP32 and FP16 storage
};
template <>
struct Acc<double> {
    using type = double;
};

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    using type = double __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<float> {
    using type = float __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<_Float16> {
    using type = _Float16 __attribute__((ext_vector_type(2)));
};

}  // namespace pp
