// Host-side metadata: boxes, box arrays, the multigrid hierarchy and the
// ghost-exchange copy tags.  Boxes are index-space rectangles with inclusive
// corners ("Box" in the paper's "Basic data structures").
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "tables.hpp"

namespace amrmg {

struct IBox {
  int lo[3], hi[3];
};

inline int ext(const IBox& b, int d) { return b.hi[d] - b.lo[d] + 1; }
inline bool ok(const IBox& b) { return b.hi[0] >= b.lo[0] && b.hi[1] >= b.lo[1] && b.hi[2] >= b.lo[2]; }
inline int64_t volume(const IBox& b) { return ok(b) ? int64_t(ext(b, 0)) * ext(b, 1) * ext(b, 2) : 0; }
inline IBox grow(const IBox& b, int g) {
  IBox r;
  for (int d = 0; d < 3; ++d) { r.lo[d] = b.lo[d] - g; r.hi[d] = b.hi[d] + g; }
  return r;
}
inline IBox shifted(const IBox& b, const int s[3]) {
  IBox r;
  for (int d = 0; d < 3; ++d) { r.lo[d] = b.lo[d] + s[d]; r.hi[d] = b.hi[d] + s[d]; }
  return r;
}
inline IBox intersect(const IBox& a, const IBox& b) {
  IBox r;
  for (int d = 0; d < 3; ++d) {
    r.lo[d] = a.lo[d] > b.lo[d] ? a.lo[d] : b.lo[d];
    r.hi[d] = a.hi[d] < b.hi[d] ? a.hi[d] : b.hi[d];
  }
  return r;
}
inline int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
inline IBox coarsen(const IBox& b, int r) {
  IBox c;
  for (int d = 0; d < 3; ++d) { c.lo[d] = floordiv(b.lo[d], r); c.hi[d] = floordiv(b.hi[d], r); }
  return c;
}
inline bool same(const IBox& a, const IBox& b) {
  for (int d = 0; d < 3; ++d)
    if (a.lo[d] != b.lo[d] || a.hi[d] != b.hi[d]) return false;
  return true;
}

struct CopyTag {
  int dst, src;
  IBox region;   // destination cells
  int shift[3];  // source cell = destination cell - shift
};

// Box array checks: non-empty boxes inside the domain, pairwise disjoint and,
// when require_cover, covering the domain.  Pairwise disjointness uses the
// same hash bins as the copy tags.  Returns false with a message on failure.
bool validate_boxes(const std::vector<IBox>& boxes, const IBox& domain, bool require_cover,
                    std::string* err);

// Copy tags of the ghost exchange, found with a uniform hash of the boxes:
// each box goes to the bin of its low corner (bin edge = largest box edge),
// built in O(N); the candidates for a grown destination box are the boxes
// in the few bins its range can reach, so listing every tag costs O(n).
// Sorted canonically by (dst, src, shift, region lo).
std::vector<CopyTag> copy_tags(const std::vector<IBox>& boxes, const IBox& domain,
                               const int periodic[3], int ngrow);

// Device copy items for the ghost exchange of a MultiFab with the given
// ngrow, per-box element offsets (of the grown arrays) and ncomp components,
// split into chunks of FB_CHUNK cells.
void make_fb_tables(const std::vector<IBox>& boxes, const IBox& domain, const int periodic[3],
                    int ngrow, const std::vector<int64_t>& offsets, int ncomp,
                    std::vector<FbTag>& tags, std::vector<FbChunk>& chunks);

// Box arrays of the multigrid levels.  Level l+1 = level l coarsened by 2,
// taken while every edge of every box is even and half of it is at least
// min_bottom_edge.  With aggregate, once that stops and the boxes cover the
// domain, the level is replaced by the single domain box (merged) and
// coarsening continues under the same rule.
struct LevelBoxes {
  std::vector<IBox> boxes;
  IBox domain;
  bool merged;  // true: this level's single box is the merged domain
};
std::vector<LevelBoxes> hierarchy(const std::vector<IBox>& boxes, const IBox& domain,
                                  int min_bottom_edge, bool aggregate);

// Thread-local error message used by mg_last_error.
void set_error(const std::string& msg);
const char* last_error();

}  // namespace amrmg
