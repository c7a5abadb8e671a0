// Plan selection by the learned cost model (filled in with the tuner).
#include "internal.h"

namespace pm {

Plan learned_plan(long lc, int pidx, bool* ok) {
  (void)lc;
  (void)pidx;
  *ok = false;
  return Plan();
}

}  // namespace pm
