// float32 exchange pipelines (one per supported grid size).
#include "exchange_kernels.hpp"

namespace hfx {
namespace {
// FusedPipeline<T, N, W, pencil threads, tile, z fwd, z inv,
//               plane threads, x fwd, x inv, y fwd, y inv>
using P24 = FusedPipeline<float, 24, 16, 64, 8, Sched<4, 6>, Sched<6, 4>, 144, Sched<4, 6>,
                          Sched<6, 4>, Sched<4, 6>, Sched<6, 4>>;
using P64 = FusedPipeline<float, 64, 16, 128, 8, Sched<8, 8>, Sched<8, 8>, 256, Sched<8, 8>,
                          Sched<8, 8>, Sched<8, 8>, Sched<8, 8>>;
using P72 = FusedPipeline<float, 72, 16, 144, 8, Sched<8, 9>, Sched<9, 8>, 216, Sched<8, 9>,
                          Sched<9, 8>, Sched<8, 9>, Sched<9, 8>>;
using P80 = FusedPipeline<float, 80, 16, 160, 8, Sched<8, 10>, Sched<10, 8>, 320, Sched<8, 10>,
                          Sched<10, 8>, Sched<8, 10>, Sched<10, 8>>;
using P96 = FusedPipeline<float, 96, 16, 192, 8, Sched<8, 12>, Sched<12, 8>, 384, Sched<8, 12>,
                          Sched<12, 8>, Sched<8, 12>, Sched<12, 8>>;
using P108 = FusedPipeline<float, 108, 16, 192, 8, Sched<12, 9>, Sched<9, 12>, 324, Sched<12, 9>,
                           Sched<9, 12>, Sched<12, 9>, Sched<9, 12>>;
using P120 = FusedPipeline<float, 120, 16, 240, 8, Sched<8, 15>, Sched<15, 8>, 480, Sched<10, 12>,
                           Sched<12, 10>, Sched<10, 12>, Sched<12, 10>>;
using P128 = FusedPipeline<float, 128, 16, 256, 8, Sched<8, 16>, Sched<16, 8>, 512, Sched<8, 16>,
                           Sched<16, 8>, Sched<8, 16>, Sched<16, 8>>;
}  // namespace

const Variant* variants_f32(int* count) {
  static const Variant v[] = {
      P24::describe("f32-n24"),   P64::describe("f32-n64"),   P72::describe("f32-n72"),
      P80::describe("f32-n80"),   P96::describe("f32-n96"),   P108::describe("f32-n108"),
      P120::describe("f32-n120"), P128::describe("f32-n128"),
  };
  *count = (int)(sizeof(v) / sizeof(v[0]));
  return v;
}

}  // namespace hfx
