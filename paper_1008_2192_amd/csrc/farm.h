// The tile farm and its work functions (the paper's framework, Sections 6.3 and 7).
//
// A work function is a struct that declares what the farm needs to know about it:
//   kList        false: one FP32 output per pixel (an image, like a cleaned subimage);
//                true : a variable number of SourceRec records (the paper's example of
//                actors returning structures instead of subimages);
//   radius(args) its dependency radius: how far from a pixel it may read, and so the
//                border a partition into independent subimages must give it for an
//                exact result (the farm itself reads neighbours straight from the
//                frame, which is resident in HBM);
//   pixel() or candidate() + find(): the per-pixel computation (list functions pass
//                every pixel through the cheap candidate() test and run find() only on
//                the candidates, compacted, so that whole waves do the expensive part);
//   kNeighbours + neighbours(): optionally, a necessary condition on the four direct
//                neighbours that the scan applies where it holds them (others come
//                as -inf).
// The farm cuts the frame into tile_h x tile_w rectangles and hands them to a
// persistent set of waves through atomic tickets, as CRBLASTER's director hands
// subimages to free actors; adding a work function means adding one struct and one
// dispatch line, nothing else in the farm changes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace crb {

constexpr int kWorkLacosmic = 0, kWorkPoisson = 1, kWorkWaiter = 2, kWorkSources = 3;
constexpr int kMaxWorkRadius = 8;        // largest radius a work function may declare
constexpr int kFarmQueues = 32;          // ticket counters (one tile range each)
constexpr int kFarmCandidates = 1024;    // candidates a wave collects before running them
constexpr int kFarmWaveRecords = 128;    // records a wave buffers before moving them

struct WorkArgs {
    unsigned long long seed;   // POISSON: generator key
    long long wall_khz;        // WAITER: rate of the wall-clock counter
    float threshold, sky;      // SOURCES: peak threshold, level subtracted in the sums
    int r, a;                  // SOURCES: peak window radius, aperture radius
};

// One SOURCES record; the layout of crb_source (40 bytes).
struct SourceRec {
    int y, x;
    float peak;
    int npix;
    double flux, sy, sx;
};

// Declared dependency radius of a work function (host side); -1 for an unknown kind.
int work_radius(int kind, const WorkArgs &a, int niter);

// Clears the kFarmQueues ticket counters and, if count is not null, the record counter.
hipError_t launch_farm_reset(unsigned int *tickets, unsigned long long *count, hipStream_t s);
// Runs work function `kind` over the frame with `workers` persistent waves (actors).
// Image kinds write out_img (H x W); list kinds append to out_list (at most capacity
// records are stored, *count receives the total).  The tickets (and *count) must be zero.
hipError_t launch_farm(int kind, const WorkArgs &args, const float *in, int H, int W,
                       int workers, int tile_h, int tile_w, float *out_img,
                       SourceRec *out_list, long long capacity, unsigned long long *count,
                       unsigned int *tickets, hipStream_t s);

}  // namespace crb
