// Registry of the compiled transform lengths (one translation unit per length).
#include <vector>

#include "fft_args.h"
#include "fft_sizes.h"

namespace krig {

#define KRIG_DECL(a, b, c) void register_fft_##a##x##b##x##c();
KRIG_FFT_SIZES(KRIG_DECL)
KRIG_FFT_VARIANTS(KRIG_DECL)
#undef KRIG_DECL

static std::vector<FftEntry>& table() {
  static std::vector<FftEntry> t;
  return t;
}

void register_fft(const FftEntry& e) { table().push_back(e); }

void register_all_fft() {
  if (!table().empty()) return;
#define KRIG_CALL(a, b, c) register_fft_##a##x##b##x##c();
  KRIG_FFT_SIZES(KRIG_CALL)  // defaults first: find_fft returns the first form of a length
  KRIG_FFT_VARIANTS(KRIG_CALL)
#undef KRIG_CALL
}

const FftEntry* find_fft(int F) {
  for (const FftEntry& e : table())
    if (e.F == F) return &e;
  return nullptr;
}

int fft_variants(int F, const FftEntry** out, int cap) {
  int k = 0;
  for (const FftEntry& e : table())
    if (e.F == F) {
      if (k < cap) out[k] = &e;
      ++k;
    }
  return k;
}

int fft_sizes(int* out, int cap) {
  int k = 0;
  for (const FftEntry& e : table()) {
    if (k < cap) out[k] = e.F;
    ++k;
  }
  return k;
}

}  // namespace krig

namespace krig {

}  // namespace krig
