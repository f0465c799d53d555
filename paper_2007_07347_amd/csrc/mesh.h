// Host-side mesh builder of the solver library: raw polygons -> per-cell slot
// arrays in the library's (optionally RCM) order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sdugks.h"

namespace sdg {

constexpr int32_t kEmptySlot = INT32_MIN;   // padding slot of a cell with fewer faces than D

struct BcEntry {
    int32_t type;
    double rho, u, v;        // SYMMETRY: (u, v) = unit outward normal of the tag's line
};

// Everything the device needs, in the library's cell order.  Per-slot arrays
// are structure-of-arrays [D][nc]: slot s of cell c at index s*nc + c.
struct MeshBuild {
    int32_t nc = 0;        // cells
    int32_t D = 0;         // slots per cell (max polygon degree)
    int32_t n_faces = 0;   // faces after periodic gluing
    int32_t n_bfaces = 0;  // boundary (non-periodic) faces
    int32_t n_singular = 0;
    double h_min = 0, dt = 0, tau = 0;
    std::vector<int32_t> perm;    // internal index -> caller index
    std::vector<int32_t> iperm;   // caller index -> internal index
    // per cell, internal order
    std::vector<double> area, cx, cy;
    std::vector<double> ainv;     // [3][nc]: (A^-1)_xx, (A^-1)_xy, (A^-1)_yy of the LSQ normal matrix
    // per slot
    std::vector<int32_t> nbr;     // >= 0 neighbour cell; < 0: -(1 + boundary face); kEmptySlot
    std::vector<double> lnx, lny; // scaled outward normal l*n of the face, seen from this cell
    std::vector<double> rsx, rsy; // face midpoint minus this cell's centroid
    std::vector<double> rox, roy; // face midpoint (in the neighbour's frame) minus the neighbour's centroid
    std::vector<double> wx, wy;   // least-squares weight A^-1 d of the stencil point behind the slot
    std::vector<int32_t> fid;     // face behind the slot (both cells of an interior face share it); -1 empty
    // boundary faces
    std::vector<int32_t> bf_cell, bf_tag;
    std::vector<BcEntry> bcs;
    // Tiles of the fused step (empty when the two-kernel step is used).  Tile t
    // owns the contiguous internal cells [g0, g0 + nt); its local cells are
    // those, then the n1 cells of its first halo ring, then the n2 of its
    // second.  Per-tile tables, padded to the largest tile (PL = nl_max local
    // cells, PA = na_max cells of tile + first ring, PT = nt_max tile cells,
    // PF = nf_max face records):
    //   lgid [n_tiles][PL]          internal id of every local cell;
    //   ladj [n_tiles][D][PA]       neighbour behind each slot of a tile or
    //                               first-ring cell: local index >= 0, -1 empty,
    //                               -2 - tag for a boundary face of that tag;
    //   lfc  [n_tiles][D][PT]       face of each slot of a tile cell: record
    //                               index * 2, + 1 if the record is stored as
    //                               seen from the other cell; -1 empty;
    //   frec [n_tiles][3][PF][2]    one record per face of the tile's cells, as
    //                               seen from the first tile cell that has it:
    //                               rows l n, r_self, r_other of (x, y).  A face
    //                               between two tile cells is stored once; the
    //                               other cell's view is (-l n, r_other, r_self),
    //                               the exact mirror the per-slot arrays hold.
    //   lw   [n_tiles][D][PA][2]    least-squares weight (x, y) behind each slot
    //                               of a tile or first-ring cell.
    int32_t tile_T = 0, n_tiles = 0, nl_max = 0, na_max = 0, nt_max = 0, nf_max = 0;
    std::vector<int32_t> tile_hdr;   // [n_tiles][8]: g0, nt, n1, n2, 0...
    std::vector<int32_t> lgid;
    std::vector<int16_t> ladj;
    std::vector<int16_t> lfc;
    std::vector<double> frec;
    std::vector<double> lw;
    // Structured step (tensor-product quad meshes; cart == true): the cells
    // are (i, j), 0 <= i < nx, 0 <= j < ny, with corners (xs[i], ys[j]) ..
    // (xs[i+1], ys[j+1]); storage tiles of kCartTX x kCartTY cells in
    // row-major tile order, cells row-major inside each tile (the internal
    // order); ntx x nty step tiles of kCartTX x cart_tile_rows(precision).  Per
    // column i, col[i][kCartVals]: width, offsets of its left and right face
    // midpoints from its centre, least-squares weights of its left and right
    // stencil points (neighbour centre, periodic image, or the wall face
    // midpoint), inverse width; per row the same in y.  Boundary-condition
    // entry of every boundary face of the four sides (-1 where periodic):
    // side[0..nx) bottom, [nx..2nx) top, [2nx..2nx+ny) left, then right.
    bool cart = false;
    int32_t nx = 0, ny = 0, ntx = 0, nty = 0, per_x = 0, per_y = 0;
    std::vector<double> col, row;
    std::vector<int32_t> side;
};

// Storage tile of the structured step (16 x 14 cells) and the per-column /
// per-row record length.  The FP32-deviation step works on whole storage
// tiles; the forms with FP64 face arithmetic on their upper and lower halves
// (16 x 7), whose cells are contiguous too, so that their LDS (twice the
// bytes per value) stays small enough for several workgroups per CU.
constexpr int32_t kCartTX = 16, kCartTY = 14;
__host__ __device__ constexpr int32_t cart_tile_rows(int precision)
{
    return precision == SDUGKS_FP32DEV ? kCartTY : kCartTY / 2;
}
constexpr int32_t kCartVals = 8;   // width, left offset, right offset, left weight, right weight, 1/width, pad, pad
// Internal index of cell (i, j) of a structured mesh: tiles in row-major
// order, each tile's cells in rows; the last tile column and row may be
// narrower.
__host__ __device__ inline int32_t cart_index(int32_t i, int32_t j, int32_t nx, int32_t ny)
{
    const int32_t tx = i / kCartTX, ty = j / kCartTY;
    const int32_t h = ny - ty * kCartTY < kCartTY ? ny - ty * kCartTY : kCartTY;
    const int32_t w = nx - tx * kCartTX < kCartTX ? nx - tx * kCartTX : kCartTX;
    return ty * kCartTY * nx + tx * kCartTX * h + (j - ty * kCartTY) * w + (i - tx * kCartTX);
}

// Accelerator complex dies of an MI355X, each with its own L2: the fused step
// gives each a contiguous range of tiles.
constexpr int32_t kXcds = 8;
// Workgroups of a batched launch with room for cap_tiles tiles (a multiple of
// kXcds, so each XCD has the same number of tile slots).
inline int32_t batch_grid(int32_t cap_tiles) { return (cap_tiles + kXcds - 1) / kXcds * kXcds; }
// The single-instance fused step launches one workgroup per tile; workgroup b
// runs on XCD b % kXcds, so XCD x gets n / kXcds tiles, one more if
// x < n % kXcds, and takes the contiguous range that starts here.
__host__ __device__ inline int32_t xcd_range_start(int32_t n, int32_t x)
{
    return x * (n / kXcds) + (x < n % kXcds ? x : n % kXcds);
}
// Boundary-condition entries the fused step keeps in LDS (more: two-kernel step).
constexpr int32_t kMaxTileBcs = 64;
// LDS words per cell of the fused step's gradient array: the 18 components
// and one pad, so that consecutive cells fall on different LDS banks (an odd
// number of words in FP32, an odd number of word pairs in FP64).
constexpr int32_t kGradStride = 19;
// LDS bytes of one workgroup of the fused step: rho and u of every tile or
// first-ring cell and the momentum of every tile cell (FP64), fbar+ of every
// local cell and the gradient of every tile or first-ring cell (elem bytes:
// 8 FP64, 4 deviation form), then the boundary-condition table (4 doubles
// per entry).
inline size_t tile_lds_bytes(int32_t nl_max, int32_t na_max, int32_t nt_max, int32_t n_bc, size_t elem = 8)
{
    const size_t head = (3 * (size_t)na_max + 2 * (size_t)nt_max) * 8 +
                        (9 * (size_t)nl_max + kGradStride * (size_t)na_max) * elem;
    return (head + 15) / 16 * 16 + 32 * (size_t)n_bc;
}
constexpr size_t kTileLdsLimit = 64 * 1024;
constexpr int32_t kDefaultBlock = 256;   // threads of the fused step; tiles hold at most a quarter as many cells

// Returns SDUGKS_OK or an error code with a message in err.
int build_mesh(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
               MeshBuild &out, std::string &err);

}  // namespace sdg
