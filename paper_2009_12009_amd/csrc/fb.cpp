// Stand-alone ghost exchange of a MultiFab ("Operations on a level") and the
// copy-tag listing.  Exchange plans are cached per (boxes, layout, geometry,
// device), as the paper caches its communication metadata ("Communication"):
// the hash intersection runs once per distinct MultiFab layout, and every
// later exchange is a single fused copy launch.
#include <hip/hip_runtime_api.h>

#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/amrmg.h"
#include "host.hpp"
#include "kernels.hpp"

using namespace amrmg;

namespace {

struct FbPlan {
  std::vector<FbTag> tags;
  std::vector<FbChunk> chunks;
  FbTag* d_tags = nullptr;
  FbChunk* d_chunks = nullptr;
  int device = 0;
};

std::mutex g_mtx;
std::map<std::string, std::unique_ptr<FbPlan>> g_cache;

template <typename T>
void put(std::string& k, const T& v) {
  k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}

IBox to_ibox(const mg_box_t& b) {
  IBox r;
  for (int d = 0; d < 3; ++d) { r.lo[d] = b.lo[d]; r.hi[d] = b.hi[d]; }
  return r;
}

}  // namespace

extern "C" {

int mg_copy_tags(const mg_box_t* boxes, int32_t nbox, const mg_geom_t* geom, int32_t ngrow,
                 mg_copy_tag_t* out, int32_t cap, int32_t* n) {
  if (!boxes || nbox <= 0 || !geom || !n || ngrow < 0) {
    set_error("mg_copy_tags: bad argument");
    return MG_ERR_ARG;
  }
  std::vector<IBox> bx(nbox);
  for (int i = 0; i < nbox; ++i) bx[i] = to_ibox(boxes[i]);
  const IBox dom = to_ibox(geom->domain);
  std::string err;
  if (!validate_boxes(bx, dom, false, &err)) {
    set_error(err);
    return MG_ERR_INVALID_BOXARRAY;
  }
  const int per[3] = {geom->is_periodic[0] != 0, geom->is_periodic[1] != 0,
                      geom->is_periodic[2] != 0};
  const std::vector<CopyTag> t = copy_tags(bx, dom, per, ngrow);
  *n = (int32_t)t.size();
  if (!out) return MG_OK;
  if (cap < (int32_t)t.size()) {
    set_error("mg_copy_tags: capacity too small");
    return MG_ERR_ARG;
  }
  for (size_t i = 0; i < t.size(); ++i) {
    out[i].dst = t[i].dst;
    out[i].src = t[i].src;
    for (int d = 0; d < 3; ++d) {
      out[i].dst_region.lo[d] = t[i].region.lo[d];
      out[i].dst_region.hi[d] = t[i].region.hi[d];
      out[i].shift[d] = t[i].shift[d];
    }
  }
  return MG_OK;
}

}  // extern "C"

namespace {

// Argument checks shared by both exchanges; *skip = nothing to exchange.
int check_fb_args(const mg_multifab_t* mf, const mg_geom_t* geom, const char* who, bool* skip) {
  *skip = false;
  if (!mf || !geom || !mf->boxes || !mf->offsets || mf->nbox <= 0) {
    set_error(std::string(who) + ": bad argument");
    return MG_ERR_ARG;
  }
  if (mf->ixtype[0] || mf->ixtype[1] || mf->ixtype[2]) {
    set_error(std::string(who) + ": only cell-centred MultiFabs are supported");
    return MG_ERR_ARG;
  }
  if (mf->ngrow < 0 || mf->ncomp < 1 || (mf->dtype != MG_F64 && mf->dtype != MG_F32)) {
    set_error(std::string(who) + ": bad ngrow, ncomp or dtype");
    return MG_ERR_ARG;
  }
  if (mf->ngrow == 0) {
    *skip = true;
    return MG_OK;
  }
  if (!mf->data) {
    set_error(std::string(who) + ": data is null");
    return MG_ERR_ARG;
  }
  return MG_OK;
}

// The cached plan of this layout on device dev, built on first use (host
// tables only; the device copy is made by the caller that needs one).
int find_plan(const mg_multifab_t* mf, const mg_geom_t* geom, int dev, FbPlan** out) {
  std::string key;
  put(key, dev);
  put(key, mf->ngrow);
  put(key, mf->ncomp);
  put(key, geom->domain);
  for (int d = 0; d < 3; ++d) put(key, (int)(geom->is_periodic[d] != 0));
  put(key, mf->nbox);
  key.append(reinterpret_cast<const char*>(mf->boxes), sizeof(mg_box_t) * mf->nbox);
  key.append(reinterpret_cast<const char*>(mf->offsets), sizeof(int64_t) * mf->nbox);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) {
    *out = it->second.get();
    return MG_OK;
  }
  std::vector<IBox> bx(mf->nbox);
  for (int i = 0; i < mf->nbox; ++i) bx[i] = to_ibox(mf->boxes[i]);
  const IBox dom = to_ibox(geom->domain);
  std::string err;
  if (!validate_boxes(bx, dom, false, &err)) {
    set_error(err);
    return MG_ERR_INVALID_BOXARRAY;
  }
  const int per[3] = {geom->is_periodic[0] != 0, geom->is_periodic[1] != 0,
                      geom->is_periodic[2] != 0};
  std::vector<int64_t> offs(mf->offsets, mf->offsets + mf->nbox);
  std::unique_ptr<FbPlan> p(new FbPlan());
  make_fb_tables(bx, dom, per, mf->ngrow, offs, mf->ncomp, p->tags, p->chunks);
  p->device = dev;
  *out = p.get();
  g_cache[key] = std::move(p);
  return MG_OK;
}

hipError_t launch_plan(const mg_multifab_t* mf, hipStream_t st, const FbTag* tags,
                       const FbChunk* chunks, int nchunks) {
  if (mf->dtype == MG_F64)
    return launch_fill_boundary<double>(st, tags, chunks, nchunks, static_cast<double*>(mf->data),
                                        mf->ncomp);
  return launch_fill_boundary<float>(st, tags, chunks, nchunks, static_cast<float*>(mf->data),
                                     mf->ncomp);
}

// Byte offset of the chunk table behind the tag table in the static scratch.
size_t chunk_offset(size_t ntags) { return (sizeof(FbTag) * ntags + 255) & ~size_t(255); }

}  // namespace

extern "C" {

int fill_boundary(mg_multifab_t* mf, const mg_geom_t* geom, void* hip_stream) {
  bool skip = false;
  int rc = check_fb_args(mf, geom, "fill_boundary", &skip);
  if (rc != MG_OK || skip) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("fill_boundary: no HIP device");
    return MG_ERR_HIP;
  }
  FbPlan* plan = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mtx);
    rc = find_plan(mf, geom, dev, &plan);
    if (rc != MG_OK) return rc;
    if (!plan->tags.empty() && !plan->d_tags) {
      FbTag* dt = nullptr;
      FbChunk* dc = nullptr;
      if (hipMalloc((void**)&dt, sizeof(FbTag) * plan->tags.size()) != hipSuccess ||
          hipMalloc((void**)&dc, sizeof(FbChunk) * plan->chunks.size()) != hipSuccess ||
          hipMemcpy(dt, plan->tags.data(), sizeof(FbTag) * plan->tags.size(),
                    hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(dc, plan->chunks.data(), sizeof(FbChunk) * plan->chunks.size(),
                    hipMemcpyHostToDevice) != hipSuccess) {
        if (dt) hipFree(dt);
        if (dc) hipFree(dc);
        set_error("fill_boundary: could not upload the exchange plan");
        return MG_ERR_HIP;
      }
      plan->d_tags = dt;
      plan->d_chunks = dc;
    }
  }
  if (plan->chunks.empty()) return MG_OK;
  const hipError_t e = launch_plan(mf, static_cast<hipStream_t>(hip_stream), plan->d_tags,
                                   plan->d_chunks, (int)plan->chunks.size());
  if (e != hipSuccess) {
    set_error(std::string("fill_boundary: ") + hipGetErrorString(e));
    return MG_ERR_HIP;
  }
  return MG_OK;
}

int mg_fill_boundary_noalloc(mg_multifab_t* mf, const mg_geom_t* geom, void* hip_stream) {
  bool skip = false;
  int rc = check_fb_args(mf, geom, "mg_fill_boundary_noalloc", &skip);
  if (rc != MG_OK || skip) return rc;
  int dev = 0;
  void* scr = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || fb_scratch_address(&scr) != hipSuccess) {
    set_error("mg_fill_boundary_noalloc: no HIP device or no scratch address");
    return MG_ERR_HIP;
  }
  FbPlan* plan = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mtx);
    rc = find_plan(mf, geom, dev, &plan);
    if (rc != MG_OK) return rc;
  }
  if (plan->chunks.empty()) return MG_OK;
  const size_t coff = chunk_offset(plan->tags.size());
  const size_t need = coff + sizeof(FbChunk) * plan->chunks.size();
  if (need > kFbScratchBytes) {
    set_error("mg_fill_boundary_noalloc: the exchange plan needs " + std::to_string(need) +
              " bytes, more than the " + std::to_string(kFbScratchBytes) +
              " bytes of static scratch; use fill_boundary");
    return MG_ERR_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  unsigned char* base = static_cast<unsigned char*>(scr);
  hipError_t e = hipMemcpyAsync(base, plan->tags.data(), sizeof(FbTag) * plan->tags.size(),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + coff, plan->chunks.data(), sizeof(FbChunk) * plan->chunks.size(),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = launch_plan(mf, st, reinterpret_cast<const FbTag*>(base),
                    reinterpret_cast<const FbChunk*>(base + coff), (int)plan->chunks.size());
  if (e != hipSuccess) {
    set_error(std::string("mg_fill_boundary_noalloc: ") + hipGetErrorString(e));
    return MG_ERR_HIP;
  }
  return MG_OK;
}

int mg_fill_boundary(mg_multifab_t* mf, const mg_geom_t* geom, void* hip_stream) {
  return fill_boundary(mf, geom, hip_stream);
}

void mg_release_caches(void) {
  std::lock_guard<std::mutex> lk(g_mtx);
  if (!g_cache.empty()) hipDeviceSynchronize();
  for (auto& kv : g_cache) {
    if (kv.second->d_tags) hipFree(kv.second->d_tags);
    if (kv.second->d_chunks) hipFree(kv.second->d_chunks);
  }
  g_cache.clear();
}

}  // extern "C"
