// Host metadata: box-array validation, the multigrid hierarchy and the
// hash-binned box intersection that produces the ghost-exchange copy tags
// (the paper's "Communication" section: an O(N) hash over the global boxes,
// then O(n) work to list the source/destination pairs).
#include "host.hpp"

#include <algorithm>
#include <cstring>
#include <tuple>
#include <unordered_map>

namespace amrmg {

namespace {

thread_local std::string g_err;

// Uniform bins over index space; bin edge = the largest box edge along d, so a
// box intersecting a query range has its low corner in a bin no further than
// one bin below the range's low bin.
struct BoxHash {
  int bsz[3];
  std::unordered_map<int64_t, std::vector<int>> bins;

  static int64_t key(int a, int b, int c) {
    // 21 bits per coordinate, offset so negative bin indices stay distinct
    const int64_t o = 1 << 20;
    return ((int64_t(a) + o) << 42) | ((int64_t(b) + o) << 21) | (int64_t(c) + o);
  }

  explicit BoxHash(const std::vector<IBox>& boxes) {
    for (int d = 0; d < 3; ++d) bsz[d] = 1;
    for (const IBox& b : boxes)
      for (int d = 0; d < 3; ++d) bsz[d] = std::max(bsz[d], ext(b, d));
    bins.reserve(boxes.size() * 2);
    for (int i = 0; i < (int)boxes.size(); ++i) {
      const IBox& b = boxes[i];
      bins[key(floordiv(b.lo[0], bsz[0]), floordiv(b.lo[1], bsz[1]), floordiv(b.lo[2], bsz[2]))]
          .push_back(i);
    }
  }

  // indices of boxes that may intersect q (a superset; caller intersects)
  void candidates(const IBox& q, std::vector<int>& out) const {
    out.clear();
    int blo[3], bhi[3];
    for (int d = 0; d < 3; ++d) {
      blo[d] = floordiv(q.lo[d], bsz[d]) - 1;
      bhi[d] = floordiv(q.hi[d], bsz[d]);
    }
    for (int c = blo[2]; c <= bhi[2]; ++c)
      for (int b = blo[1]; b <= bhi[1]; ++b)
        for (int a = blo[0]; a <= bhi[0]; ++a) {
          auto it = bins.find(key(a, b, c));
          if (it == bins.end()) continue;
          out.insert(out.end(), it->second.begin(), it->second.end());
        }
  }
};

std::string box_str(const IBox& b) {
  char buf[160];
  snprintf(buf, sizeof(buf), "[(%d,%d,%d)-(%d,%d,%d)]", b.lo[0], b.lo[1], b.lo[2], b.hi[0], b.hi[1],
           b.hi[2]);
  return buf;
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

bool validate_boxes(const std::vector<IBox>& boxes, const IBox& domain, bool require_cover,
                    std::string* err) {
  if (boxes.empty()) {
    *err = "empty box array";
    return false;
  }
  if (!ok(domain)) {
    *err = "empty domain";
    return false;
  }
  int64_t cells = 0;
  for (size_t i = 0; i < boxes.size(); ++i) {
    const IBox& b = boxes[i];
    if (!ok(b)) {
      *err = "box " + std::to_string(i) + " is empty " + box_str(b);
      return false;
    }
    if (!same(intersect(b, domain), b)) {
      *err = "box " + std::to_string(i) + " " + box_str(b) + " lies outside the domain " +
             box_str(domain);
      return false;
    }
    cells += volume(b);
  }
  BoxHash hash(boxes);
  std::vector<int> cand;
  for (size_t i = 0; i < boxes.size(); ++i) {
    hash.candidates(boxes[i], cand);
    for (int j : cand) {
      if (j == (int)i) continue;
      if (ok(intersect(boxes[i], boxes[j]))) {
        *err = "boxes " + std::to_string(std::min<int>(i, j)) + " and " +
               std::to_string(std::max<int>(i, j)) + " intersect";
        return false;
      }
    }
  }
  if (require_cover && cells != volume(domain)) {
    *err = "box array does not cover the domain (" + std::to_string(cells) + " of " +
           std::to_string(volume(domain)) + " cells)";
    return false;
  }
  return true;
}

std::vector<CopyTag> copy_tags(const std::vector<IBox>& boxes, const IBox& domain,
                               const int periodic[3], int ngrow) {
  std::vector<CopyTag> tags;
  BoxHash hash(boxes);
  int L[3];
  for (int d = 0; d < 3; ++d) L[d] = ext(domain, d);
  std::vector<int> cand;
  for (int bi = 0; bi < (int)boxes.size(); ++bi) {
    const IBox gb = grow(boxes[bi], ngrow);
    for (int sx = -1; sx <= 1; ++sx)
      for (int sy = -1; sy <= 1; ++sy)
        for (int sz = -1; sz <= 1; ++sz) {
          const int sv[3] = {sx, sy, sz};
          bool skip = false;
          int s[3];
          for (int d = 0; d < 3; ++d) {
            if (sv[d] != 0 && !periodic[d]) skip = true;
            s[d] = sv[d] * L[d];
          }
          if (skip) continue;
          // source boxes S with (S + s) n gb non-empty <=> S n (gb - s) non-empty
          int ms[3] = {-s[0], -s[1], -s[2]};
          hash.candidates(shifted(gb, ms), cand);
          for (int si : cand) {
            if (si == bi && s[0] == 0 && s[1] == 0 && s[2] == 0) continue;
            IBox r = intersect(gb, shifted(boxes[si], s));
            if (!ok(r)) continue;
            CopyTag t;
            t.dst = bi;
            t.src = si;
            t.region = r;
            for (int d = 0; d < 3; ++d) t.shift[d] = s[d];
            tags.push_back(t);
          }
        }
  }
  std::sort(tags.begin(), tags.end(), [](const CopyTag& a, const CopyTag& b) {
    return std::make_tuple(a.dst, a.src, a.shift[0], a.shift[1], a.shift[2], a.region.lo[0],
                           a.region.lo[1], a.region.lo[2]) <
           std::make_tuple(b.dst, b.src, b.shift[0], b.shift[1], b.shift[2], b.region.lo[0],
                           b.region.lo[1], b.region.lo[2]);
  });
  return tags;
}

void make_fb_tables(const std::vector<IBox>& boxes, const IBox& domain, const int periodic[3],
                    int ngrow, const std::vector<int64_t>& offsets, int ncomp,
                    std::vector<FbTag>& tags, std::vector<FbChunk>& chunks) {
  tags.clear();
  chunks.clear();
  const std::vector<CopyTag> ct = copy_tags(boxes, domain, periodic, ngrow);
  for (const CopyTag& t : ct) {
    const IBox& D = boxes[t.dst];
    const IBox& S = boxes[t.src];
    const int dnx = ext(D, 0) + 2 * ngrow, dny = ext(D, 1) + 2 * ngrow;
    const int snx = ext(S, 0) + 2 * ngrow, sny = ext(S, 1) + 2 * ngrow;
    int dl[3], sl[3];
    for (int d = 0; d < 3; ++d) {
      dl[d] = t.region.lo[d] - (D.lo[d] - ngrow);
      sl[d] = t.region.lo[d] - t.shift[d] - (S.lo[d] - ngrow);
    }
    FbTag g;
    g.dsy = dnx;
    g.dsz = dnx * dny;
    g.ssy = snx;
    g.ssz = snx * sny;
    g.dst_base = offsets[t.dst] + dl[0] + (long long)dl[1] * g.dsy + (long long)dl[2] * g.dsz;
    g.src_base = offsets[t.src] + sl[0] + (long long)sl[1] * g.ssy + (long long)sl[2] * g.ssz;
    g.dst_cstride = ncomp > 1 ? (long long)dnx * dny * (ext(D, 2) + 2 * ngrow) : 0;
    g.src_cstride = ncomp > 1 ? (long long)snx * sny * (ext(S, 2) + 2 * ngrow) : 0;
    g.nx = ext(t.region, 0);
    g.ny = ext(t.region, 1);
    g.ncell = (int)volume(t.region);
    g.pad = 0;
    const int ti = (int)tags.size();
    tags.push_back(g);
    for (int s = 0; s < g.ncell; s += FB_CHUNK) chunks.push_back({ti, s});
  }
}

static bool coarsenable(const std::vector<IBox>& boxes, const IBox& domain, int min_edge) {
  for (const IBox& b : boxes)
    for (int d = 0; d < 3; ++d) {
      int e = ext(b, d);
      if (e % 2 != 0 || e / 2 < min_edge || ((b.lo[d] % 2) + 2) % 2 != 0) return false;
    }
  for (int d = 0; d < 3; ++d)
    if (ext(domain, d) % 2 != 0 || ((domain.lo[d] % 2) + 2) % 2 != 0) return false;
  return true;
}

std::vector<LevelBoxes> hierarchy(const std::vector<IBox>& boxes, const IBox& domain,
                                  int min_bottom_edge, bool aggregate) {
  std::vector<LevelBoxes> levels;
  levels.push_back({boxes, domain, false});
  if (min_bottom_edge < 1) min_bottom_edge = 1;
  while (true) {
    const LevelBoxes& cur = levels.back();
    if (coarsenable(cur.boxes, cur.domain, min_bottom_edge)) {
      LevelBoxes nxt;
      for (const IBox& b : cur.boxes) nxt.boxes.push_back(coarsen(b, 2));
      nxt.domain = coarsen(cur.domain, 2);
      nxt.merged = false;
      levels.push_back(nxt);
      continue;
    }
    if (!aggregate || cur.boxes.size() == 1) break;
    // merge: every box must split into whole 2x2x2 blocks, the level must cover
    // its domain, and the merged domain must pass the coarsening rule
    bool even = true;
    int64_t cells = 0;
    for (const IBox& b : cur.boxes) {
      cells += volume(b);
      for (int d = 0; d < 3; ++d)
        if (((b.lo[d] % 2) + 2) % 2 != 0 || ext(b, d) % 2 != 0) even = false;
    }
    if (!even || cells != volume(cur.domain)) break;
    if (!coarsenable({cur.domain}, cur.domain, min_bottom_edge)) break;
    LevelBoxes nxt;
    nxt.domain = coarsen(cur.domain, 2);
    nxt.boxes = {nxt.domain};
    nxt.merged = true;
    levels.push_back(nxt);
  }
  return levels;
}

}  // namespace amrmg
