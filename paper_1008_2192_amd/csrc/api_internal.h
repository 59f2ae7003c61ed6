// Internal helpers shared by the C ABI translation units of libcrb.
#pragma once

#include "../../include/crb.h"
#include "farm.h"
#include "kernels.h"

namespace crb {

// Byte offsets of one frame's workspace pieces (256-byte aligned).
struct FrameWs {
    size_t codes, list, nnew, listlen, dirty, tile_first, tile_new, total;
};

crb_status fail(crb_status st, const char *fmt, ...);
crb_status ok();
crb_status hip_status(hipError_t e, const char *what);
crb_status check_frame_args(int32_t H, int32_t W, float gain, float readnoise, float sky,
                            float sigclip, float sigfrac, float objlim, int32_t niter);
crb_status check_buffers(const float *img, const float *clean, const uint8_t *mask,
                         size_t npix);
FrameWs ws_layout(int32_t H, int32_t W);
DevFrame make_devframe(const float *img, float *J, uint8_t *mask, char *ws, const FrameWs &L,
                       int32_t H, int32_t W, float gain, float readnoise, float sky,
                       float sigclip, float sigfrac, float objlim, int32_t niter, int32_t flags);
int replace_grid(size_t npix);

}  // namespace crb
