// Entry points not built yet: they validate nothing and report UNSUPPORTED.
#include "ctv.h"
#include "ctv_host.hpp"

using namespace ctv;

extern "C" {
ctv_status pr_workspace_size(const pr_params*, int32_t, int32_t, size_t*) { return fail(CTV_ERR_UNSUPPORTED, "not built"); }
ctv_status pr_prox_grad(const pr_params*, int32_t, int32_t, const float*, float*, float*, void*, size_t, ctv_stream_t) { return fail(CTV_ERR_UNSUPPORTED, "not built"); }
ctv_status ctv_fft2(int32_t, int32_t, int32_t, const float*, float*, int32_t, ctv_stream_t) { return fail(CTV_ERR_UNSUPPORTED, "not built"); }
ctv_status pr_forward(const pr_params*, int32_t, int32_t, const float*, float*, void*, size_t, ctv_stream_t) { return fail(CTV_ERR_UNSUPPORTED, "not built"); }
ctv_status pr_gradient(const pr_params*, int32_t, int32_t, const float*, const float*, float*, float*, void*, size_t, ctv_stream_t) { return fail(CTV_ERR_UNSUPPORTED, "not built"); }
}
