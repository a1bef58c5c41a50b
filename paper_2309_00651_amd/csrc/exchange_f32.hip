// float32 exchange pipelines (one per supported grid size).
#include "exchange_kernels.hpp"

namespace hfx {
namespace {
// FusedPipeline<T, N, W, tile, z fwd, z inv, plane threads, x fwd, x inv,
//               y fwd, y inv [, swizzle, pair_fwd threads, inv_acc threads]>
// Plane threads: the plane takes N (N + 1) * 8 bytes of LDS, so from N = 96 at
// most two planes fit in a compute unit; more threads per plane then buy the
// occupancy that hides the LDS and HBM latencies.
using P24 = FusedPipeline<float, 24, 16, 8, Sched<4, 6>, Sched<6, 4>, 144, Sched<4, 6>,
                          Sched<6, 4>, Sched<4, 6>, Sched<6, 4>>;
using P64 = FusedPipeline<float, 64, 16, 8, Sched<8, 8>, Sched<8, 8>, 256, Sched<8, 8>,
                          Sched<8, 8>, Sched<8, 8>, Sched<8, 8>>;
using P64q512 = FusedPipeline<float, 64, 16, 8, Sched<8, 8>, Sched<8, 8>, 512, Sched<8, 8>,
                              Sched<8, 8>, Sched<8, 8>, Sched<8, 8>>;
using P64r = FusedPipeline<float, 64, 16, 8, Sched<8, 8>, Sched<8, 8>, 256, Sched<8, 8>,
                           Sched<8, 8>, Sched<8, 8>, Sched<8, 8>, false, 256, 512, false, false>;
using P72 = FusedPipeline<float, 72, 16, 8, Sched<8, 9>, Sched<9, 8>, 576, Sched<8, 9>,
                          Sched<9, 8>, Sched<8, 9>, Sched<9, 8>>;
using P72q216 = FusedPipeline<float, 72, 16, 8, Sched<8, 9>, Sched<9, 8>, 216, Sched<8, 9>,
                              Sched<9, 8>, Sched<8, 9>, Sched<9, 8>>;
using P72r = FusedPipeline<float, 72, 16, 8, Sched<8, 9>, Sched<9, 8>, 576, Sched<8, 9>,
                           Sched<9, 8>, Sched<8, 9>, Sched<9, 8>, false, 256, 512, false, false>;
using P80 = FusedPipeline<float, 80, 16, 8, Sched<8, 10>, Sched<10, 8>, 640, Sched<8, 10>,
                          Sched<10, 8>, Sched<8, 10>, Sched<10, 8>>;
using P80q320 = FusedPipeline<float, 80, 16, 8, Sched<8, 10>, Sched<10, 8>, 320, Sched<8, 10>,
                              Sched<10, 8>, Sched<8, 10>, Sched<10, 8>>;
using P80r = FusedPipeline<float, 80, 16, 8, Sched<8, 10>, Sched<10, 8>, 640, Sched<8, 10>,
                           Sched<10, 8>, Sched<8, 10>, Sched<10, 8>, false, 256, 512, false, false>;
using P96 = FusedPipeline<float, 96, 16, 8, Sched<8, 12>, Sched<8, 12>, 768, Sched<8, 12>,
                          Sched<12, 8>, Sched<8, 12>, Sched<12, 8>>;
// alternatives for the autotuner (here and below): psi J block in registers
// without prefetch (-r) or in LDS with prefetch (-lp); radix-12-first inverse z; plane threads; swizzled plane LDS;
// psi I block in LDS
using P96r = FusedPipeline<float, 96, 16, 8, Sched<8, 12>, Sched<8, 12>, 768, Sched<8, 12>,
                           Sched<12, 8>, Sched<8, 12>, Sched<12, 8>, false, 256, 512, false, false>;
using P96z12 = FusedPipeline<float, 96, 16, 8, Sched<8, 12>, Sched<12, 8>, 768, Sched<8, 12>,
                             Sched<12, 8>, Sched<8, 12>, Sched<12, 8>>;
using P96q384 = FusedPipeline<float, 96, 16, 8, Sched<8, 12>, Sched<8, 12>, 384, Sched<8, 12>,
                              Sched<12, 8>, Sched<8, 12>, Sched<12, 8>>;
using P96sw = FusedPipeline<float, 96, 16, 8, Sched<8, 12>, Sched<8, 12>, 768, Sched<8, 12>,
                            Sched<12, 8>, Sched<8, 12>, Sched<12, 8>, true>;
using P96pi = FusedPipeline<float, 96, 16, 8, Sched<8, 12>, Sched<8, 12>, 768, Sched<8, 12>,
                            Sched<12, 8>, Sched<8, 12>, Sched<12, 8>, false, 512, 512, true, true,
                            true>;
// Grids whose fused plane fills a compute unit's LDS (108 to 128): one plane
// workgroup per compute unit.  Defaults: flat-load prefetching accumulation
// (inv_acc loads spread over all threads, staged in LDS) and, at 108 and 120,
// the persistent plane kernel that prefetches the next plane (at 120 with
// radix-15 first stages, which keep its registers within the budget) and an
// accumulation transform over the four grids of a tile row (psi J block in
// LDS: the larger prefetch leaves no registers for it).  Measured per K psi
// pass (ms, accumulation pass in brackets): 108^3 / 320 orbitals at 5 Ha
// 245.5 [112.2] against 251.5 [118.4] with two grids per transform (-fl2);
// 120^3 / 384 473.1 [214.5] against 483.0 [224.5]; at 128^3 / 512 four grids
// per transform were slower (468 against 414), and so was the persistent
// plane kernel (-pp: 742 against 711 for the plane pass); there the plane
// pass takes the XOR-swizzled LDS layout (the radix-8 first row stage writes
// with a stride of 8 elements, which otherwise conflicts on the LDS banks,
// 31 % of the cycles) and grid-major plane order: 709 -> 616 ms per K psi
// pass (swizzle alone 635; grid-major alone 693).  Alternatives: the earlier
// defaults (-fl: unswizzled kz-major plane; -lp: psi J block in LDS +
// prefetch; -r: registers, no prefetch), the persistent plane kernel (-pp)
// and the plane held in registers with two workgroups per compute unit (-h2,
// 702 ms: it spills 17 registers).
using P108 = FusedPipeline<float, 108, 16, 8, Sched<12, 9>, Sched<9, 12>, 972, Sched<12, 9>,
                           Sched<9, 12>, Sched<12, 9>, Sched<9, 12>, false, 256, 1024, true, true,
                           false, true, 108, 4>;
using P108fl2 = FusedPipeline<float, 108, 16, 8, Sched<12, 9>, Sched<9, 12>, 972, Sched<12, 9>,
                              Sched<9, 12>, Sched<12, 9>, Sched<9, 12>, false, 256, 1024, false,
                              true, false, true, 108, 1>;
using P108lp = FusedPipeline<float, 108, 16, 8, Sched<12, 9>, Sched<9, 12>, 972, Sched<12, 9>,
                             Sched<9, 12>, Sched<12, 9>, Sched<9, 12>>;
using P108r = FusedPipeline<float, 108, 16, 8, Sched<12, 9>, Sched<9, 12>, 972, Sched<12, 9>,
                            Sched<9, 12>, Sched<12, 9>, Sched<9, 12>, false, 256, 1024, false,
                            false>;
using P120 = FusedPipeline<float, 120, 16, 8, Sched<8, 15>, Sched<15, 8>, 960, Sched<15, 8>,
                           Sched<8, 15>, Sched<15, 8>, Sched<8, 15>, false, 256, 1024, true, true,
                           false, true, 120, 4>;
using P120fl2 = FusedPipeline<float, 120, 16, 8, Sched<8, 15>, Sched<15, 8>, 960, Sched<15, 8>,
                              Sched<8, 15>, Sched<15, 8>, Sched<8, 15>, false, 256, 1024, false,
                              true, false, true, 120, 1>;
using P120r = FusedPipeline<float, 120, 16, 8, Sched<8, 15>, Sched<15, 8>, 960, Sched<10, 12>,
                            Sched<12, 10>, Sched<10, 12>, Sched<12, 10>>;
using P120lp = FusedPipeline<float, 120, 16, 8, Sched<8, 15>, Sched<15, 8>, 960, Sched<10, 12>,
                             Sched<12, 10>, Sched<10, 12>, Sched<12, 10>, false, 256, 1024, true,
                             true>;
using P128 = FusedPipeline<float, 128, 16, 8, Sched<8, 16>, Sched<16, 8>, 1024, Sched<8, 16>,
                           Sched<16, 8>, Sched<8, 16>, Sched<16, 8>, true, 256, 1024, false, true,
                           false, false, 128, 1, HalfZ<64>::type, 1, true>;
using P128fl = FusedPipeline<float, 128, 16, 8, Sched<8, 16>, Sched<16, 8>, 1024, Sched<8, 16>,
                             Sched<16, 8>, Sched<8, 16>, Sched<16, 8>, false, 256, 1024, false, true,
                             false, false, 128, 1>;
// plane in registers with a half-plane LDS buffer: two plane workgroups of
// 512 threads per compute unit (k_plane_h2)
using P128h2 = FusedPipeline<float, 128, 16, 8, Sched<8, 16>, Sched<16, 8>, 512, Sched<8, 16>,
                             Sched<16, 8>, Sched<8, 16>, Sched<16, 8>, false, 256, 1024, false, true,
                             false, false, 128, 1, HalfZ<64>::type, 2>;
using P128r = FusedPipeline<float, 128, 16, 8, Sched<8, 16>, Sched<16, 8>, 1024, Sched<8, 16>,
                            Sched<16, 8>, Sched<8, 16>, Sched<16, 8>>;
using P128lp = FusedPipeline<float, 128, 16, 8, Sched<8, 16>, Sched<16, 8>, 1024, Sched<8, 16>,
                             Sched<16, 8>, Sched<8, 16>, Sched<16, 8>, false, 256, 1024, true,
                             true>;
using P128pp = FusedPipeline<float, 128, 16, 8, Sched<8, 16>, Sched<16, 8>, 1024, Sched<8, 16>,
                             Sched<16, 8>, Sched<8, 16>, Sched<16, 8>, false, 256, 1024, false,
                             false, false, true>;
// slab cells (n x n x nz): z transforms of length nz, planes of n x n
using P24x48 = FusedPipeline<float, 24, 16, 8, Sched<4, 12>, Sched<12, 4>, 144, Sched<4, 6>,
                             Sched<6, 4>, Sched<4, 6>, Sched<6, 4>, false, 256, 512, true, true,
                             false, false, 48>;
using P64x128 = FusedPipeline<float, 64, 16, 8, Sched<8, 16>, Sched<16, 8>, 256, Sched<8, 8>,
                              Sched<8, 8>, Sched<8, 8>, Sched<8, 8>, false, 256, 1024, false, false,
                              false, false, 128>;
}  // namespace

const Variant* variants_f32(int* count) {
  static const Variant v[] = {
      P24::describe("f32-n24"),
      P64::describe("f32-n64"),
      P64q512::describe("f32-n64-q512"),
      P64r::describe("f32-n64-r"),
      P72::describe("f32-n72"),
      P72q216::describe("f32-n72-q216"),
      P72r::describe("f32-n72-r"),
      P80::describe("f32-n80"),
      P80q320::describe("f32-n80-q320"),
      P80r::describe("f32-n80-r"),
      P96::describe("f32-n96"),
      P96r::describe("f32-n96-r"),
      P96z12::describe("f32-n96-z12"),
      P96q384::describe("f32-n96-q384"),
      P96sw::describe("f32-n96-sw"),
      P96pi::describe("f32-n96-pi"),
      P108::describe("f32-n108"),
      P108fl2::describe("f32-n108-fl2"),
      P108lp::describe("f32-n108-lp"),
      P108r::describe("f32-n108-r"),
      P120::describe("f32-n120"),
      P120fl2::describe("f32-n120-fl2"),
      P120r::describe("f32-n120-r"),
      P120lp::describe("f32-n120-lp"),
      P128::describe("f32-n128"),
      P128fl::describe("f32-n128-fl"),
      P128r::describe("f32-n128-r"),
      P128lp::describe("f32-n128-lp"),
      P128pp::describe("f32-n128-pp"),
      P128h2::describe("f32-n128-h2"),
      P24x48::describe("f32-n24x48"),
      P64x128::describe("f32-n64x128"),
  };
  *count = (int)(sizeof(v) / sizeof(v[0]));
  return v;
}

}  // namespace hfx
