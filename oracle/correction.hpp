// Oracle: tag of a learned flux correction (TEST INFRASTRUCTURE ONLY).  The
// solver takes one optional correction: the per-face network (mlp.hpp) or
// the convolutional network over the face images (cnn.hpp).
#pragma once

namespace orc {

enum CorrectionKind { CORR_MLP = 1, CORR_CNN = 2 };

struct Correction {
  int kind = 0;
};

}  // namespace orc
