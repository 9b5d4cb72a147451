// kernels_static_f64.hip -- FP64 specialised pass kernels (see static_table.hpp)
#include "static_table.hpp"

namespace hom {
namespace {
using T = double;
// Rader variants of the prime lengths 127 and 61, registered first (the
// default where no tuned choice exists; the chirp-z variants below stay and
// the tuner picks per pass)
RegCol<T, P127R, 127, 8, 256> c127r;
RegRow<T, P127R, 127, 2, 4, 256> r127r_2;
RegRow<T, P127R, 127, 3, 4, 256> r127r_3;
RegCol<T, P61R, 31, 16, 256> c61r;
RegRow<T, P61R, 31, 2, 8, 256> r61r_2;
RegRow<T, P61R, 31, 3, 8, 256> r61r_3;
RegCol<T, P1023, 1023, 2, 256> c1023;
RegCol<T, P1023, 1023, 4, 512> c1023w;
RegCol<T, P1023, 1023, 1, 128> c1023n1;
RegCol<T, P255, 255, 8, 256> c255;
RegCol<T, P255, 255, 4, 256> c255n;
RegCol<T, P127, 127, 8, 256> c127;
RegCol<T, P63, 63, 16, 256> c63;
RegCol<T, P31, 31, 16, 256> c31;
RegCol<T, P15, 15, 16, 256> c15;
RegCol<T, P253, 127, 8, 256> c253;
RegCol<T, P253, 127, 4, 256> c253n;
RegCol<T, P125, 63, 16, 256> c125;
RegCol<T, P61, 31, 16, 256> c61;
RegCol<T, P29, 15, 16, 256> c29;
RegCol<T, P509, 255, 4, 512> c509;
RegColCP<T, P1023, 1023, 1, 2, 256> x1023_1;
RegColCP<T, P255, 255, 4, 3, 192> x255_4;
RegColCP<T, P255, 255, 8, 3, 384> x255_8;
RegColCP<T, P253, 127, 4, 3, 192> x253_4;
RegColCP<T, P127, 127, 4, 3, 256> x127_4;
RegRow<T, P1023, 1023, 2, 1, 256> r1023_2;
RegRow<T, P1023, 1023, 2, 2, 512> r1023_2w;
RegRow<T, P1023, 1023, 2, 1, 128> r1023_2n;
RegRow<T, P1023, 1023, 3, 1, 256> r1023_3;
RegRow<T, P255, 255, 2, 4, 256> r255_2;
RegRow<T, P255, 255, 3, 4, 256> r255_3;
// six Mandel components (3-D elasticity)
RegRow<T, P255, 255, 6, 2, 256> r255_6;
RegRow<T, P127, 127, 2, 4, 256> r127_2;
RegRow<T, P127, 127, 3, 4, 256> r127_3;
RegRow<T, P63, 63, 2, 8, 256> r63_2;
RegRow<T, P63, 63, 3, 8, 256> r63_3;
RegRow<T, P31, 31, 2, 8, 256> r31_2;
RegRow<T, P31, 31, 3, 8, 256> r31_3;
RegRow<T, P15, 15, 2, 8, 256> r15_2;
RegRow<T, P15, 15, 3, 8, 256> r15_3;
RegRow<T, P253, 127, 2, 4, 256> r253_2;
RegRow<T, P253, 127, 3, 4, 256> r253_3;
RegRow<T, P125, 63, 2, 8, 256> r125_2;
RegRow<T, P125, 63, 3, 8, 256> r125_3;
RegRow<T, P61, 31, 2, 8, 256> r61_2;
RegRow<T, P61, 31, 3, 8, 256> r61_3;
RegRow<T, P29, 15, 2, 8, 256> r29_2;
RegRow<T, P29, 15, 3, 8, 256> r29_3;
RegRow<T, P509, 255, 2, 2, 512> r509_2;
RegRow<T, P509, 255, 3, 1, 256> r509_3;
// plain passes with the register pipeline (two-stage plans)
RegColReg2<T, P255, 255, 8, 256> g255;
RegColReg2<T, P253, 127, 8, 256> g253;
RegColReg2<T, P63, 63, 8, 128> g63;
// two spectra between the first- and middle-axis passes (3-D)
RegColR2<T, P255, 255, 8, 128> e255;
RegMid2<T, P255, 255, 8, 128> m255;
RegColR2<T, P253, 127, 8, 128> e253;
RegMid2<T, P253, 127, 8, 128> m253;
RegColR2<T, P63, 63, 8, 128> e63;
RegMid2<T, P63, 63, 8, 128> m63;
// last-axis passes of one wave per workgroup
RegRow<T, P255, 255, 3, 1, 64> r255_3q;
RegRow<T, P253, 127, 3, 1, 64> r253_3q;
}  // namespace
}  // namespace hom
