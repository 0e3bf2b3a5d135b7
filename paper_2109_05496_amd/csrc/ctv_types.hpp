// Types shared by host and device code of the HIP path (internal).
#pragma once

namespace ctv {

enum Kind { K1I = 0, K1A = 1, K2I = 2, K2A = 3 };
enum Constr { C_NONE = 0, C_MOD = 1 };

constexpr int kMaxFuse = 16;

// Row-sweep tile (fgp_sweep.hip): 8 waves, 4-row windows per wave, at most 10
// fused iterations (its LDS ring holds T + 2 rows per lane), segments of
// kSweepSegRows[i] output rows. TileShape::waves == kSweepShape selects it.
constexpr int kSweepWaves = 8;
constexpr int kSweepRows = 4;
constexpr int kSweepMaxFuse = 10;
constexpr int kSweepShape = -2;

// Smallest positive lambda accepted: 1/(8 lambda^2) (the backward's step
// derivative) and the squared dual norms stay far from float32 overflow.
constexpr float kMinLambda = 1e-12f;

// Radii of the dual balls: type-I uses 1; type-II uses alpha for the real
// plane's dual (r) and 1 - alpha for the imaginary plane's dual (s).
struct Radii {
  float ra, ra2, sa, sa2;
};

}  // namespace ctv
