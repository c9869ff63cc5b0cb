// Factor-graph engine instantiated for double state and arithmetic.
#include "graph_engine.h"

namespace admmg {

EngineBase* make_engine_f64(int device) {
  auto* e = new Engine<double>();
  e->device = device;
  return e;
}

}  // namespace admmg
