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

int fill_boundary(mg_multifab_t* mf, const mg_geom_t* geom, void* hip_stream) {
  if (!mf || !geom || !mf->boxes || !mf->offsets || mf->nbox <= 0) {
    set_error("fill_boundary: bad argument");
    return MG_ERR_ARG;
  }
  if (mf->ixtype[0] || mf->ixtype[1] || mf->ixtype[2]) {
    set_error("fill_boundary: only cell-centred MultiFabs are supported");
    return MG_ERR_ARG;
  }
  if (mf->ngrow < 0 || mf->ncomp < 1 || (mf->dtype != MG_F64 && mf->dtype != MG_F32)) {
    set_error("fill_boundary: bad ngrow, ncomp or dtype");
    return MG_ERR_ARG;
  }
  if (mf->ngrow == 0) return MG_OK;
  if (!mf->data) {
    set_error("fill_boundary: data is null");
    return MG_ERR_ARG;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("fill_boundary: no HIP device");
    return MG_ERR_HIP;
  }
  std::string key;
  put(key, dev);
  put(key, mf->ngrow);
  put(key, mf->ncomp);
  put(key, geom->domain);
  for (int d = 0; d < 3; ++d) put(key, (int)(geom->is_periodic[d] != 0));
  put(key, mf->nbox);
  key.append(reinterpret_cast<const char*>(mf->boxes), sizeof(mg_box_t) * mf->nbox);
  key.append(reinterpret_cast<const char*>(mf->offsets), sizeof(int64_t) * mf->nbox);

  FbPlan* plan = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mtx);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      plan = it->second.get();
    } else {
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
      if (!p->tags.empty()) {
        if (hipMalloc((void**)&p->d_tags, sizeof(FbTag) * p->tags.size()) != hipSuccess ||
            hipMalloc((void**)&p->d_chunks, sizeof(FbChunk) * p->chunks.size()) != hipSuccess ||
            hipMemcpy(p->d_tags, p->tags.data(), sizeof(FbTag) * p->tags.size(),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->d_chunks, p->chunks.data(), sizeof(FbChunk) * p->chunks.size(),
                      hipMemcpyHostToDevice) != hipSuccess) {
          if (p->d_tags) hipFree(p->d_tags);
          if (p->d_chunks) hipFree(p->d_chunks);
          set_error("fill_boundary: could not upload the exchange plan");
          return MG_ERR_HIP;
        }
      }
      plan = p.get();
      g_cache[key] = std::move(p);
    }
  }
  if (plan->chunks.empty()) return MG_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  if (mf->dtype == MG_F64)
    e = launch_fill_boundary<double>(st, plan->d_tags, plan->d_chunks, (int)plan->chunks.size(),
                                     static_cast<double*>(mf->data), mf->ncomp);
  else
    e = launch_fill_boundary<float>(st, plan->d_tags, plan->d_chunks, (int)plan->chunks.size(),
                                    static_cast<float*>(mf->data), mf->ncomp);
  if (e != hipSuccess) {
    set_error(std::string("fill_boundary: ") + hipGetErrorString(e));
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
