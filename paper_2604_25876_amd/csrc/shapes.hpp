// shapes.hpp -- the tile shapes compiled for the fused sweep, per precision.
//
// An entry X(NWI, NWH, HPT, COLS, PER_CU, COST): NWI interior waves (one output site per
// lane, NWI x 64 / COLS rows of COLS columns), NWH halo waves whose lanes hold HPT halo
// positions each, PER_CU blocks resident on one CU (LDS and registers), and the relative
// time of one output site and plane of an item in a full round of the chip (measured at
// 256^3) that the default tile choice weighs shapes by.  A build may define its own lists
// (one shape per precision for a quick build, say) before this header.
#pragma once

#ifndef SKYR_SHAPES_F64
#define SKYR_SHAPES_F64(X) X(4, 4, 1, 16, 1, 1.0) X(4, 4, 1, 32, 1, 1.02) X(6, 2, 2, 32, 1, 0.95)
#endif
#ifndef SKYR_SHAPES_F32
#define SKYR_SHAPES_F32(X) X(8, 4, 1, 32, 1, 1.0) X(6, 2, 2, 32, 2, 2.0) X(12, 4, 1, 32, 1, 0.9)
#endif
