// Factor-graph engine instantiated for float state and arithmetic.
#include "graph_engine.h"

namespace admmg {

EngineBase* make_engine_f32(int device) {
  auto* e = new Engine<float>();
  e->device = device;
  return e;
}

}  // namespace admmg
