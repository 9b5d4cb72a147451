// kernels_static_f32.hip -- FP32 specialised pass kernels (see static_table.hpp)
#include "static_table.hpp"

namespace hom {
namespace {
using T = float;
// Rader variants of the prime lengths 127 and 61, registered first (the
// default where no tuned choice exists; the chirp-z variants below stay and
// the tuner picks per pass)
RegCol<T, P127R, 127, 16, 256> c127r;
RegCol<T, P127R, 127, 8, 256> c127rn;
RegRow<T, P127R, 127, 2, 8, 256> r127r_2;
RegRow<T, P127R, 127, 3, 8, 256> r127r_3;
RegCol<T, P61R, 31, 16, 256> c61r;
RegRow<T, P61R, 31, 2, 8, 256> r61r_2;
RegRow<T, P61R, 31, 3, 8, 256> r61r_3;
// columns: plan, trial length, W, workgroup size
RegCol<T, P1023, 1023, 4, 256> c1023;
RegCol<T, P1023, 1023, 8, 512> c1023w;
RegCol<T, P1023, 1023, 2, 128> c1023n2;
RegCol<T, P1023, 1023, 1, 64> c1023n1;
RegCol<T, P255, 255, 16, 256> c255;
RegCol<T, P255, 255, 8, 256> c255n;
RegCol<T, P255, 255, 4, 128> c255n4;
RegCol<T, P127, 127, 16, 256> c127;
RegCol<T, P63, 63, 16, 256> c63;
RegCol<T, P31, 31, 16, 256> c31;
RegCol<T, P15, 15, 16, 256> c15;
RegCol<T, P253, 127, 16, 256> c253;
RegCol<T, P253, 127, 8, 256> c253n;
RegCol<T, P125, 63, 16, 256> c125;
RegCol<T, P61, 31, 16, 256> c61;
RegCol<T, P29, 15, 16, 256> c29;
RegCol<T, P509, 255, 8, 512> c509;
// columns, all components per transform: plan, trial length, W, components,
// workgroup size
RegColCP<T, P1023, 1023, 4, 2, 512> x1023_4;
RegColCP<T, P1023, 1023, 2, 2, 256> x1023_2;
RegColCP<T, P1023, 1023, 1, 2, 128> x1023_1;
RegColCP<T, P1023, 1023, 3, 2, 384> x1023_3;
RegColCP<T, P1023, 1023, 2, 2, 512> x1023_2w;
RegColCP<T, P1023, 1023, 1, 2, 256> x1023_1w;
// first (radix-31) stage on the matrix cores
RegColCP<T, P1023, 1023, 2, 2, 256, true> x1023_2m;
RegColCP<T, P1023, 1023, 1, 2, 128, true> x1023_1m;
RegColCP<T, P1023, 1023, 4, 2, 512, true> x1023_4m;
RegColCP<T, P255, 255, 8, 3, 384> x255_8;
RegColCP<T, P255, 255, 4, 3, 192> x255_4;
RegColCP<T, P255, 255, 16, 3, 768> x255_16;
RegColCP<T, P255, 255, 8, 2, 256> x255_8d2;
RegColCP<T, P253, 127, 8, 3, 320> x253_8;
RegColCP<T, P253, 127, 4, 3, 192> x253_4;
RegColCP<T, P127, 127, 8, 3, 256> x127_8;
RegColCP<T, P63, 63, 16, 3, 256> x63_16;
// rows: plan, trial length, components, row pairs, workgroup size
RegRow<T, P1023, 1023, 2, 2, 256> r1023_2;
RegRow<T, P1023, 1023, 2, 4, 512> r1023_2w;
RegRow<T, P1023, 1023, 2, 1, 128> r1023_2n;
RegRow<T, P1023, 1023, 2, 3, 384> r1023_2m;
RegRow<T, P1023, 1023, 2, 1, 256> r1023_2nw;
RegRow<T, P1023, 1023, 2, 2, 512> r1023_2w2;
RegRow<T, P1023, 1023, 2, 1, 128, true> r1023_2nm;
RegRow<T, P1023, 1023, 2, 2, 256, true> r1023_2mm;
RegRow<T, P1023, 1023, 3, 2, 512> r1023_3;
RegRow<T, P255, 255, 2, 8, 256> r255_2;
RegRow<T, P255, 255, 3, 8, 512> r255_3;
RegRow<T, P255, 255, 3, 4, 256> r255_3n;
RegRow<T, P127, 127, 2, 8, 256> r127_2;
RegRow<T, P127, 127, 3, 8, 512> r127_3;
RegRow<T, P63, 63, 2, 8, 256> r63_2;
RegRow<T, P63, 63, 3, 8, 256> r63_3;
RegRow<T, P31, 31, 2, 8, 256> r31_2;
RegRow<T, P31, 31, 3, 8, 256> r31_3;
RegRow<T, P15, 15, 2, 8, 256> r15_2;
RegRow<T, P15, 15, 3, 8, 256> r15_3;
RegRow<T, P253, 127, 2, 8, 256> r253_2;
RegRow<T, P253, 127, 3, 8, 512> r253_3;
RegRow<T, P253, 127, 3, 4, 256> r253_3n;
RegRow<T, P125, 63, 2, 8, 256> r125_2;
RegRow<T, P125, 63, 3, 8, 256> r125_3;
RegRow<T, P61, 31, 2, 8, 256> r61_2;
RegRow<T, P61, 31, 3, 8, 256> r61_3;
RegRow<T, P29, 15, 2, 8, 256> r29_2;
RegRow<T, P29, 15, 3, 8, 256> r29_3;
RegRow<T, P509, 255, 2, 4, 512> r509_2;
RegRow<T, P509, 255, 3, 2, 512> r509_3;
// first (radix-17 / radix-23) stage on the matrix cores
RegCol<T, P255, 255, 16, 256, true> c255m;
RegCol<T, P255, 255, 8, 256, true> c255nm;
RegCol<T, P253, 127, 16, 256, true> c253m;
RegCol<T, P253, 127, 8, 256, true> c253nm;
RegColCP<T, P255, 255, 8, 3, 384, true> x255_8m;
RegColCP<T, P253, 127, 4, 3, 192, true> x253_4m;
RegRow<T, P255, 255, 3, 4, 256, true> r255_3nm;
RegRow<T, P253, 127, 3, 4, 256, true> r253_3nm;
// wider workgroups on 16-column tiles: fewer positions per thread
RegCol<T, P255, 255, 16, 384, false, 3> c255w3;
RegCol<T, P253, 127, 16, 384> c253w3;
// 1023-point tiles with more waves per workgroup (fewer rounds per stage)
RegColCP<T, P1023, 1023, 2, 2, 384, true> x1023_2m3;
RegColCP<T, P1023, 1023, 1, 2, 192, true> x1023_1m3;
RegRow<T, P1023, 1023, 2, 1, 192, true> r1023_2nm3;
RegRow<T, P1023, 1023, 2, 1, 256, true> r1023_2nm4;
RegColCP<T, P1023, 1023, 2, 2, 320, true> x1023_2m5;
RegRow<T, P1023, 1023, 2, 1, 320, true> r1023_2nm5;
RegRow<T, P1023, 1023, 2, 1, 384, true> r1023_2nm6;
// wide tiles: longer contiguous runs along the last axis per row of the
// axis-0 / axis-1 passes (fewer, larger workgroups)
// projection with every component's tile loaded up front
RegProjPre<T, P255, 255, 16, 256> p255pre;
RegProjPre<T, P255, 255, 8, 256> p255pre8;
RegProjPre<T, P253, 127, 16, 256> p253pre;
// 16-column tiles with 512 threads: half the positions per thread
RegCol<T, P255, 255, 16, 512> c255t512;
// last-axis pass with the load cases of a row tile on consecutive workgroups
RegRow<T, P255, 255, 3, 4, 256, false, true> r255_3i;
// six Mandel components (3-D elasticity)
RegRow<T, P255, 255, 6, 2, 256> r255_6;
RegRow<T, P253, 127, 3, 4, 256, false, true> r253_3i;
RegRow<T, P1023, 1023, 2, 1, 320, true, true> r1023_2i;
// plain passes with the register pipeline (two-stage plans)
RegColReg2<T, P255, 255, 16, 256> g255;
RegColReg2<T, P255, 255, 8, 128> g255n;
RegColReg2<T, P255, 255, 16, 512> g255t;
RegColReg2<T, P253, 127, 16, 512> g253t;
RegColReg2<T, P253, 127, 16, 256> g253;
RegColReg2<T, P63, 63, 16, 128> g63;
// 3-D first-axis expansion and projection with the register pipeline
// (256 threads: four workgroups per CU; 320 and 512 threads, one
// butterfly per thread in both stages, ran slower)
RegColR2<T, P255, 255, 16, 256> e255;
RegColR2<T, P253, 127, 16, 256> e253;
RegColR2<T, P63, 63, 16, 128> e63;
RegBExpand<T, P255, 255, 16, 256> b255;
// 32-column tiles (256-byte row segments), 512 threads: 255-point expansion
// 164 -> 132 us, projection 182 -> 177 us, middle forward 230 -> 225 us (the
// middle inverse ran slower, 204 -> 238 us; the tuner picks per pass)
RegColR2<T, P255, 255, 32, 512> e255w;
RegMid2<T, P255, 255, 32, 512> m255w;
RegColR2<T, P253, 127, 32, 512> e253w;
RegMid2<T, P253, 127, 32, 512> m253w;
// last-axis flux pass with the three load cases of a row tile together
// (coefficient rows read once): 412 -> 366 us on the 253-point Ga axis; on the
// 255-point GaNi axis (twice the bytes per line) 428-517 against 364 us
RegRowMulti<T, P253, 127, 3, 2, 256, 3> q253_3;
RegMid2<T, P255, 255, 16, 256> m255;
RegMid2<T, P253, 127, 16, 256> m253;
RegMid2<T, P63, 63, 16, 128> m63;
RegMid2<T, P255, 255, 16, 512> m255t;
RegMid2<T, P253, 127, 16, 512> m253t;
// last-axis passes of one wave per workgroup: its barriers hold no other
// wave, and more workgroups fit per CU under the LDS budget
RegRow<T, P255, 255, 3, 2, 128> r255_3h;
RegRow<T, P255, 255, 3, 1, 64> r255_3q;
RegRow<T, P253, 127, 3, 1, 64> r253_3q;
RegRow<T, P1023, 1023, 2, 1, 64> r1023_2q;
}  // namespace
}  // namespace hom
