// Kernel argument blocks and host launchers of the HIP path (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctv_types.hpp"

namespace ctv {

constexpr int kPlainChunk = 32;  // images per plain launch (per-image lambda lives in kernargs)

struct FgpPlainArgs {
  const float* b;        // chunk base, [chunk][m][n] complex64
  const uint8_t* mask;   // [m][n] or nullptr
  const float* st_in;    // [chunk][2][m][n][4] or nullptr (cold start)
  float* st_out;         // same layout or nullptr
  float* x;              // [chunk][m][n] complex64 or nullptr
  int m, n;
  int tiles_x, tiles_y;
  int halo;
  int T;
  Radii R;
  float beta[kMaxFuse];  // beta[i] = (t_k - 1)/t_{k+1} for the i-th fused iteration k
  float lam[kPlainChunk];
  float c[kPlainChunk];  // 1 / (8 lambda)
  float* r_hist;         // 8 x 8 column tile only: states [T][chunk][2][m][n][4] whose plane 1
                         // receives r after each fused iteration (output pixels), or nullptr
  long long r_hist_stride;  // floats from one iteration's state to the next
  const int* live;       // column and row-sweep tiles: [0] = L, [1 .. L] = the tiles (of one image) to
                         // run, or nullptr for all; the grid stays one workgroup per tile of the chunk
  int sweep_rows;        // row-sweep tile: output rows of a tile (a segment); 0 otherwise
};

// Persistent dataflow form of the plain path (8 x 8 column tile): one launch
// runs every fused step of a chunk of images. Tasks (step, image, tile) are
// handed out in that order from an atomic ticket; a task waits until the 3 x 3
// neighbouring tiles of the same image have finished the previous step (the
// halo is smaller than a tile's output, so no other tile overlaps), then runs
// the same tile function as the per-step launches. After the compute steps one
// more step with no iterations writes x (Eq. 18) and, if asked, the state.
constexpr int kFlowMaxIters = 480;  // iterations per launch (the momentum table lives in kernargs)

struct FgpFlowArgs {
  const float* b;         // chunk base, complex64
  const uint8_t* mask;    // [m][n] or nullptr
  const float* st_in;     // initial state or nullptr (cold start)
  float* buf0;            // ping-pong states [chunk][2][m][n][4]: step s reads buf[s % 2] (buf0 at
  float* buf1;            // s = 0 unless st_in) and writes buf[(s + 1) % 2]
  float* st_out;          // final state or nullptr
  float* x;               // complex64 output
  int* counter;           // ticket counter, zero at launch
  int* done;              // [chunk][tiles]: steps completed, zero at launch
  int* err;               // set to 1 if a dependency wait gave up; the epilogue then writes NaN
  int preset_err;         // test hook: raise *err at launch, so every wait gives up at once
  int m, n, tiles_x, tiles_y, batch;
  int halo;               // = T for every step
  int T, T_last, steps;   // fused iterations per step (last compute step: T_last), compute steps
  Radii R;
  float lam[kPlainChunk];
  float c[kPlainChunk];
  float beta[kFlowMaxIters];  // beta[i]: momentum of the i-th iteration of this launch
};
hipError_t launch_fgp_flow(const FgpFlowArgs& a, int kind, int constr, hipStream_t s);

// Images that fit in one 8 x 8 column tile (m, n <= 64) have no neighbouring
// tiles, hence no halo: one workgroup per image runs up to kFlowMaxIters
// iterations in a single launch.
struct FgpSingleArgs {
  const float* b;         // chunk base, complex64
  const uint8_t* mask;    // [m][n] or nullptr
  const float* st_in;     // [chunk][2][m][n][4] or nullptr (cold start)
  float* st_out;          // same layout or nullptr
  float* x;               // complex64 output or nullptr
  int m, n, T;
  Radii R;
  float lam[kPlainChunk];
  float c[kPlainChunk];
  float beta[kFlowMaxIters];
};
hipError_t launch_fgp_single(const FgpSingleArgs& a, int kind, int constr, int batch, hipStream_t s);
// Ints of flow bookkeeping (counter, error flag, done flags) for `batch` images of m x n at halo h.
long long flow_ints(int batch, int m, int n, int h);

struct BatchImage {
  long long offset;          // first pixel in the packed image buffers
  long long support_offset;  // byte offset of the mask, -1 = none
  int m, n;
  int kind;
  int iters;                 // 0 for lambda = 0 (x = P_C(b))
  float lam, c;
  Radii R;
};

struct BatchTile {
  int image, tx, ty;
  int flag;                  // index of the tile's live flag, or -1 (image without a support: always runs)
};

// One (image, tiling) pair of a batched plan whose tiles are scanned for
// liveness (images with a support): flags [flag_base, flag_base + tiles_x *
// tiles_y). zero_st: this scan stores zeros at the image's dead pixels in both
// state buffers (one pair per image); zero_x: it stores x = 0 in dead tiles
// (the tiling of the image's last step).
struct BatchGeom {
  int image, halo, tiles_x, tiles_y, flag_base, zero_st, zero_x, pad;
};

struct BatchScanArgs {
  const BatchImage* images;
  const BatchGeom* geoms;
  const int* geo_of;        // [nflags] the pair each flag belongs to
  const uint8_t* support;
  float* st0;               // the two packed state buffers
  float* st1;
  float* x;
  int* flags;
  int rows;                 // region rows of the tile shape (column tiles)
  int sweep_oh;             // row-sweep tile: output rows of a tile (region rows then sweep_oh + 2 halo); 0 otherwise
};

struct BatchCompactArgs {
  const BatchTile* tiles;   // every step's tiles
  const int* step_offset;   // [steps]
  const int* step_count;    // [steps]
  const int* flags;
  int* lists;               // same indexing as tiles: step s's list at lists[step_offset[s]]
  int* counts;              // [steps]
};
const void* batched_scan_kernel_ptr();
const void* batched_compact_kernel_ptr();

struct FgpBatchedArgs {
  const BatchTile* tiles;   // this step's tiles
  int ntiles;
  const BatchImage* images;
  const float* beta_table;  // beta_table[k] = (t_k - 1)/t_{k+1}, k >= 1
  const float* b;
  const uint8_t* support;
  const float* st_in;       // packed [2 * pixels][4] per image at 2 * offset
  float* st_out;
  float* x;
  int k0;                   // iterations completed before this step
  int T;                    // iterations fused in this step
  const int* live;          // this step's tiles to run (indices into tiles) or nullptr = all
  const int* live_count;
  int sweep_rows;           // row-sweep tile: output rows of a tile; 0 for the column tiles
};

// Tile shape of the plain kernels: waves > 0 selects the column-register tile
// (waves wave64s, rows_per_thread consecutive rows each); waves == 0 selects the
// LDS tile with 4 waves and rows_per_thread * 4 region rows; waves ==
// kSweepShape the row-sweep tile with rows_per_thread output rows per tile.
struct TileShape {
  int waves;
  int rows_per_thread;
  bool sweep() const { return waves == kSweepShape; }
  // region rows without the halo (column / LDS tiles) or output rows (row sweep)
  int rows() const { return sweep() ? rows_per_thread : (waves > 0 ? waves : 4) * rows_per_thread; }
  // output rows of a tile at halo H
  int out_rows(int H) const { return sweep() ? rows_per_thread : rows() - 2 * H; }
  // workgroup size
  int threads() const { return sweep() ? kSweepWaves * 64 : (waves > 0 ? waves : 4) * 64; }
};
bool valid_tile_shape(const TileShape& ts);
// Batched kernel for a column-register tile shape (8x8, 8x4 or 16x4) or the
// row-sweep tile, else nullptr.
const void* fgp_batched_kernel_ptr(int constr, const TileShape& ts);

hipError_t launch_fgp_plain(const FgpPlainArgs& a, int kind, int constr, const TileShape& ts, int batch,
                            hipStream_t s);
hipError_t launch_fgp_sweep(const FgpPlainArgs& a, int kind, int constr, int batch, hipStream_t s);
const void* fgp_sweep_batched_kernel_ptr(int constr);

hipError_t launch_zero_f4(float* p, long long count_f4, hipStream_t s);

// Live tiles of a support for one tiling (see live_scan_kernel): flags[tiles]
// scratch, then live[0] = L and live[1 .. L] the live tiles in increasing order.
struct LiveScanArgs {
  const uint8_t* mask;   // [m][n]
  int m, n;
  int halo, rows;        // the tiling: regions of rows x 64 with this halo
  int tiles_x, tiles_y;
  int* flags;
  int zero_st;           // store zeros at dead output pixels of st0 and st1
  float* st0;            // chunk bases of the two state buffers [batch][2][m][n][4]
  float* st1;
  float* x;              // chunk base of x [batch][m][n] complex64 (zeroed in dead tiles) or nullptr
  int batch;
};
hipError_t launch_live_tiles(const LiveScanArgs& a, int* live, hipStream_t s);
hipError_t launch_project_c(const float* b, const uint8_t* mask, float* x, long long px, int batch,
                            int constr, hipStream_t s);
struct GapArgs {
  float lam[kPlainChunk];
};
hipError_t launch_gap(const float* x, const float* state, int m, int n, int batch, int kind,
                      Radii R, const GapArgs& lam, double* partial, int blocks_per_img,
                      double* gap, hipStream_t s);

}  // namespace ctv
