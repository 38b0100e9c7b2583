// Types shared by the device kernels and the host code of the library.
#pragma once
#include <stdint.h>

namespace stereo_dev {

constexpr int kMaxPairs = 8;  // pairs per launch of the integer path

// Image pointers of the pairs of one launch (passed by value to the kernels).
struct PairPtrs {
  const uint8_t* left[kMaxPairs];
  const uint8_t* right[kMaxPairs];
  int16_t* out[kMaxPairs];
};

}  // namespace stereo_dev
