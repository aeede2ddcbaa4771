// FP64 engines (plain one-field-at-a-time path), one per supported grid side.
#include "pgx_engine.hpp"

namespace pgx {
EngineBase* make_engine_f64(const PlanCfg& c) {
  switch (c.N) {
    case 64: return new Engine<double, 64>(c);
    case 128: return new Engine<double, 128>(c);
    case 256: return new Engine<double, 256>(c);
    case 512: return new Engine<double, 512>(c);
    case 1024: return new Engine<double, 1024>(c);
    default: return nullptr;
  }
}
}  // namespace pgx
