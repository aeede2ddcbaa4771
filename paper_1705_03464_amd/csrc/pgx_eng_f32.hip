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
size_t memory_bound_f32(const PlanCfg& c, int64_t n, int64_t P, bool spectra) {
  switch (c.N) {
    case 64: return Engine<float, 64>::memory_bound(c, n, P, spectra);
    case 128: return Engine<float, 128>::memory_bound(c, n, P, spectra);
    case 256: return Engine<float, 256>::memory_bound(c, n, P, spectra);
    case 512: return Engine<float, 512>::memory_bound(c, n, P, spectra);
    case 1024: return Engine<float, 1024>::memory_bound(c, n, P, spectra);
    default: return 0;
  }
}
}  // namespace pgx
