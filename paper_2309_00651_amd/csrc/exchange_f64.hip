// float64 exchange pipelines.  Planes of up to 96^2 points fit in LDS in
// float64; larger grids split the plane pass into x rows and y columns.
#include "exchange_kernels.hpp"

namespace hfx {
namespace {
// Plane threads: a float64 plane of 64^2 points or more leaves room for one
// or two workgroups per compute unit, so the plane kernels take 8 threads
// per row (the alternatives with 4 per row are kept for the autotuner).
using P24 = FusedPipeline<double, 24, 16, 8, Sched<4, 6>, Sched<6, 4>, 144, Sched<4, 6>,
                          Sched<6, 4>, Sched<4, 6>, Sched<6, 4>>;
using P64 = FusedPipeline<double, 64, 16, 8, Sched<8, 8>, Sched<8, 8>, 512, Sched<8, 8>,
                          Sched<8, 8>, Sched<8, 8>, Sched<8, 8>>;
using P72 = FusedPipeline<double, 72, 16, 8, Sched<8, 9>, Sched<9, 8>, 576, Sched<8, 9>,
                          Sched<9, 8>, Sched<8, 9>, Sched<9, 8>>;
using P80 = FusedPipeline<double, 80, 16, 8, Sched<8, 10>, Sched<10, 8>, 640, Sched<8, 10>,
                          Sched<10, 8>, Sched<8, 10>, Sched<10, 8>>;
using P96 = FusedPipeline<double, 96, 16, 8, Sched<8, 12>, Sched<12, 8>, 768, Sched<8, 12>,
                          Sched<12, 8>, Sched<8, 12>, Sched<12, 8>>;
using P64q256 = FusedPipeline<double, 64, 16, 8, Sched<8, 8>, Sched<8, 8>, 256, Sched<8, 8>,
                              Sched<8, 8>, Sched<8, 8>, Sched<8, 8>>;
using P72q216 = FusedPipeline<double, 72, 16, 8, Sched<8, 9>, Sched<9, 8>, 216, Sched<8, 9>,
                              Sched<9, 8>, Sched<8, 9>, Sched<9, 8>>;
using P80q320 = FusedPipeline<double, 80, 16, 8, Sched<8, 10>, Sched<10, 8>, 320, Sched<8, 10>,
                              Sched<10, 8>, Sched<8, 10>, Sched<10, 8>>;
using P96q384 = FusedPipeline<double, 96, 16, 8, Sched<8, 12>, Sched<12, 8>, 384, Sched<8, 12>,
                              Sched<12, 8>, Sched<8, 12>, Sched<12, 8>>;
using P96z8 = FusedPipeline<double, 96, 16, 8, Sched<8, 12>, Sched<8, 12>, 768, Sched<8, 12>,
                            Sched<12, 8>, Sched<8, 12>, Sched<12, 8>>;
// three-stage inverse z: the accumulation kernel stays below 160 registers
// (12 x 8 and 10 x 8 spill 14 without a cutoff)
using P96s3 = FusedPipeline<double, 96, 16, 8, Sched<8, 12>, Sched<8, 4, 3>, 768, Sched<8, 12>,
                            Sched<12, 8>, Sched<8, 12>, Sched<12, 8>>;
using P80s3 = FusedPipeline<double, 80, 16, 8, Sched<8, 10>, Sched<5, 4, 4>, 640, Sched<8, 10>,
                            Sched<10, 8>, Sched<8, 10>, Sched<10, 8>>;
// slab cells (n x n x nz); the 128-point inverse z takes 8 x 4 x 4, with
// which its accumulation kernel does not spill (see below)
using P24x48 = FusedPipeline<double, 24, 16, 8, Sched<4, 12>, Sched<12, 4>, 144, Sched<4, 6>,
                             Sched<6, 4>, Sched<4, 6>, Sched<6, 4>, false, 384, 384, false, false,
                             false, false, 48>;
using P64x128 = FusedPipeline<double, 64, 16, 8, Sched<8, 16>, Sched<8, 4, 4>, 512, Sched<8, 8>,
                              Sched<8, 8>, Sched<8, 8>, Sched<8, 8>, false, 512, 512, false, false,
                              false, false, 128>;
// SplitPipeline<T, N, W, column threads, tile, z fwd, z inv, rows per wg,
//               row threads, x fwd, x inv, y fwd, y inv>
// The inverse z schedules are the ones whose accumulation kernel fits the 256
// registers of its two waves per SIMD without spills (a spilled register of
// the loop is written to scratch every iteration, and the grid stream evicts
// those lines): 12 x 9, 12 x 10 and 8 x 4 x 4 (the radix-16 stage of 16 x 8
// alone holds 64 registers of float64 values and spilled 54; 15 x 8 spilled
// 32, 9 x 12 4).
using P108 = SplitPipeline<double, 108, 16, 192, 8, Sched<12, 9>, Sched<12, 9>, 16, 192,
                           Sched<12, 9>, Sched<9, 12>, Sched<12, 9>, Sched<9, 12>>;
using P120 = SplitPipeline<double, 120, 16, 240, 8, Sched<8, 15>, Sched<12, 10>, 16, 240,
                           Sched<8, 15>, Sched<15, 8>, Sched<8, 15>, Sched<15, 8>>;
using P128 = SplitPipeline<double, 128, 16, 256, 8, Sched<8, 16>, Sched<8, 4, 4>, 16, 256,
                           Sched<8, 16>, Sched<16, 8>, Sched<8, 16>, Sched<16, 8>>;
// the earlier inverse z schedules, for the autotuner
using P108z = SplitPipeline<double, 108, 16, 192, 8, Sched<12, 9>, Sched<9, 12>, 16, 192,
                            Sched<12, 9>, Sched<9, 12>, Sched<12, 9>, Sched<9, 12>>;
using P120z = SplitPipeline<double, 120, 16, 240, 8, Sched<8, 15>, Sched<15, 8>, 16, 240,
                            Sched<8, 15>, Sched<15, 8>, Sched<8, 15>, Sched<15, 8>>;
using P128z = SplitPipeline<double, 128, 16, 256, 8, Sched<8, 16>, Sched<16, 8>, 16, 256,
                            Sched<8, 16>, Sched<16, 8>, Sched<8, 16>, Sched<16, 8>>;
}  // namespace

const Variant* variants_f64(int* count) {
  static const Variant v[] = {
      P24::describe("f64-n24"),
      P64::describe("f64-n64"),
      P64q256::describe("f64-n64-q256"),
      P72::describe("f64-n72"),
      P72q216::describe("f64-n72-q216"),
      P80::describe("f64-n80"),
      P80q320::describe("f64-n80-q320"),
      P96::describe("f64-n96"),
      P96q384::describe("f64-n96-q384"),
      P96z8::describe("f64-n96-z8"),
      P96s3::describe("f64-n96-s3"),
      P80s3::describe("f64-n80-s3"),
      P108::describe("f64-n108"),
      P108z::describe("f64-n108-z"),
      P120::describe("f64-n120"),
      P120z::describe("f64-n120-z"),
      P128::describe("f64-n128"),
      P128z::describe("f64-n128-z"),
      P24x48::describe("f64-n24x48"),
      P64x128::describe("f64-n64x128"),
  };
  *count = (int)(sizeof(v) / sizeof(v[0]));
  return v;
}

}  // namespace hfx
