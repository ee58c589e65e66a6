// Complex FP64 value as stored in device memory: interleaved (re, im).
#pragma once

namespace mfq {

struct cplx {
  double re, im;
};

}  // namespace mfq
