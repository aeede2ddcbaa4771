// FP32 engines (batched field-pair path), one per supported grid side.
#include "pgx_engine.hpp"

namespace pgx {
EngineBase* make_engine_f32(const PlanCfg& c) {
  switch (c.N) {
    case 64: return new Engine<float, 64>(c);
    case 128: return new Engine<float, 128>(c);
    case 256: return new Engine<float, 256>(c);
    case 512: return new Engine<float, 512>(c);
    case 1024: return new Engine<float, 1024>(c);
    default: return nullptr;
  }
}
}  // namespace pgx
