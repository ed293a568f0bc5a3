// Entry points not yet implemented in this build.
#include "kt_internal.hpp"

using namespace kt;

namespace kt {
kt_status select_config(Ctx* h, const kt_shape*, int32_t*) {
  return fail(h, KT_ENOTFITTED, "no selector fitted");
}
}

extern "C" {
kt_status kt_normalize(kt_handle h, const int64_t*, int32_t, int32_t, kt_norm, uint16_t*, void*) {
  return fail((Ctx*)h, KT_EUNSUPPORTED, "not implemented");
}
kt_status kt_prune_workspace_bytes(int32_t, int32_t, int32_t, int32_t, size_t*) { return KT_EUNSUPPORTED; }
kt_status kt_prune(kt_handle h, const int64_t*, int32_t, int32_t, int32_t, kt_norm, uint64_t, int32_t,
                   int32_t, void*, size_t, void*, int32_t*, int64_t*, int32_t*, int64_t*) {
  return fail((Ctx*)h, KT_EUNSUPPORTED, "not implemented");
}
kt_status kt_prune_topn(kt_handle h, const int64_t*, int32_t, int32_t, int32_t, int32_t*) {
  return fail((Ctx*)h, KT_EUNSUPPORTED, "not implemented");
}
kt_status kt_fit_selector(kt_handle h, kt_selector, const kt_shape*, const int64_t*, int32_t, int32_t,
                          const int32_t*, int32_t, const kt_mlp_opts*, void*, size_t, void*) {
  return fail((Ctx*)h, KT_EUNSUPPORTED, "not implemented");
}
kt_status kt_select(kt_handle h, const kt_shape*, int32_t*) { return fail((Ctx*)h, KT_ENOTFITTED, "no selector"); }
kt_status kt_select_batch(kt_handle h, const kt_shape*, int32_t, int32_t*, void*) {
  return fail((Ctx*)h, KT_ENOTFITTED, "no selector");
}
kt_status kt_get_tree(kt_handle h, int32_t*, int32_t*, int64_t*, int32_t*, int32_t*, int32_t*) {
  return fail((Ctx*)h, KT_ENOTFITTED, "no tree");
}
kt_status kt_save(kt_handle h, const char*) { return fail((Ctx*)h, KT_ENOTFITTED, "no selector"); }
kt_status kt_load(kt_handle h, const char*) { return fail((Ctx*)h, KT_EIO, "not implemented"); }
}
