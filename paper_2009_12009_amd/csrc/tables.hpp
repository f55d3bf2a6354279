// Plain structs shared by the host driver and the device kernels: the per-box
// table of a level, tile work items and ghost-copy items.  Everything a kernel
// needs to find a cell of a box is in these tables, so one launch covers every
// box of a level (the box-list form of "MFIter" with tiling off on the GPU).
#pragma once

#include <cstdint>

namespace amrmg {

// bcmask bits: 2*d set = the low face along d is a Dirichlet wall, 2*d+1 = the
// high face.
struct BoxInfo {
  int lo[3];
  int hi[3];
  int bcmask;
  int parent;          // box of the next coarser level that holds coarsen(this box)
  long long off_g1;    // element offset of this box in cell data with 1 ghost layer
  long long off_g0;    // ... in cell data without ghosts
  long long off_f[3];  // ... in face data of direction d (ghost-free, +1 along d)
};

// One work-group's share: a tile of one box starting at cell (x0, y0, z0).
// The tile extent is set by the launch, except for the smoother half-sweep,
// which reads its lane layout from shape when non-zero: log2(lx) in bits
// 0-3, ly in bits 4-11, planes in bits 16-31 (the tile's box class shape).
struct Tile {
  int box;
  int x0, y0, z0;
  int shape;
};

// One ghost-copy item, resolved to element offsets: region cell (i, j, k)
// (0-based inside the region) goes to dst_base + i + j*dsy + k*dsz from
// src_base + i + j*ssy + k*ssz; component c adds c*cstride.
struct FbTag {
  long long dst_base, src_base;
  long long dst_cstride, src_cstride;
  int nx, ny, ncell, pad;
  int dsy, dsz, ssy, ssz;
};

// FB_CHUNK consecutive cells of one tag, handled by one work-group.
struct FbChunk {
  int tag;
  int start;
};

constexpr int FB_CHUNK = 256;

// Write-through of a smoother update into other boxes' face ghosts: the
// valid cells lo..hi (box-local, inclusive) of a source box are the face
// ghosts of one destination box; local cell (i, j, k) goes to element
// base + i + j*sy + k*sz of the level's array.
struct WtEntry {
  int lo[3], hi[3];
  long long base;
  int sy, sz;
};

// Per source box and face (xlo, xhi, ylo, yhi, zlo, zhi): the range of its
// write-through entries.
struct WtBox {
  int first[6];
  int count[6];
};

// A block of cells of one box (box-local offsets i0, j0, k0 from the box's
// low corner, extents ni, nj, nk, at most 256 cells) on the box's boundary
// layer, where the fused sweep leaves the second colour's update to a pass
// of its own.
struct RimTile {
  int box;
  int i0, j0, k0;
  int ni, nj, nk;
  int pad;
};

// A fine ghost cell filled from the coarse level: dst (element in the fine
// array, one ghost layer) = v_C + 1/4 sum_d sigma_d (v_{C+e_d} - v_{C-e_d}) / 2.
// c and nb[] are elements of the coarse array (ghost layer 1, each in the box
// that owns the cell); nb[2d] / nb[2d+1] = low / high neighbour along d, -1
// past a Dirichlet wall (then -v_C).  sign bit d set = high half along d.
struct CfGhost {
  long long dst;
  long long c;
  long long nb[6];
  int sign;
  int pad;
};

// An uncovered coarse cell next to the fine region: its residual (element
// r_idx, ghost-free layout) gets, for each of its count coarse/fine faces,
// the coarse face term put back and the mean fine flux taken off.
struct CfCell {
  long long r_idx;
  long long phi_idx;  // element of the cell in the coarse array (ghost layer 1)
  int first, count;
};

// One coarse/fine face of a CfCell: the covered neighbour J, the coarse face,
// and the 4 fine cells of J next to the face with their ghosts in I.
struct CfFace {
  long long j_idx;     // coarse array element of J (ghost layer 1, J's own box)
  long long cb_idx;    // element of the coarse face coefficient (direction d)
  long long fv[4];     // fine array elements (ghost layer 1) of the fine cells in J
  long long fg[4];     // fine array elements of their ghosts in I
  long long fb[4];     // fine face coefficient elements (direction d)
  int d, pad;
};

}  // namespace amrmg
