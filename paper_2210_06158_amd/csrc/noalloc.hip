// dof_render_frame_noalloc: the frame pass with its scratch in a buffer the
// library owns, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The buffer is a file-scope device array: every GPU the library runs on
// holds one copy (kNoAllocScratchBytes) until the process ends.  In host code
// the array's name only stands in for it, so its device address is looked up
// once per device with hipGetSymbolAddress, on that device's first call, and
// only that address is passed on.  All calls on one GPU share the buffer and
// it keeps the last call's contents; the pass writes every plane it reads
// (counters included) before reading it, so nothing needs clearing between
// calls.  Calls that overlap on one GPU (two streams, two threads) race on
// the buffer.
#include <mutex>

#include "dof_internal.h"

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)DOF_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];   // device address of `scratch` on each device (nullptr: not looked up yet)

}  // namespace

extern "C" dof_status dof_render_frame_noalloc(dof_scene *scene, const dof_camera *cam, const dof_lens *lens,
                                               const dof_gbuffer *gb, const dof_history_io *hist, const dof_params *p,
                                               const dof_frame_out *out, void *stream)
{
    if (!cam || !p) return dof_render_frame(scene, cam, lens, gb, hist, p, out, nullptr, 0, stream);   // its checks report
    if (p->struct_size == sizeof(dof_params) && p->timing)
        return dof::set_error(DOF_E_UNSUPPORTED, "dof_render_frame_noalloc: params.timing needs event objects; use dof_render_frame");
    size_t need = 0;
    dof_status st = dof_frame_scratch_bytes(cam->width, cam->height, p, &need);
    if (st != DOF_OK) return st;
    if (need > kNoAllocScratchBytes)
        return dof::set_error(DOF_E_UNSUPPORTED,
                                "dof_render_frame_noalloc: this frame needs %zu bytes of scratch, the library's buffer "
                                "holds %zu (use dof_render_frame with a caller buffer)",
                                need, kNoAllocScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dof::set_error(DOF_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return dof::set_error(DOF_E_UNSUPPORTED, "device %d out of range", dev);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_ptr[dev]) {
            void *a = nullptr;
            e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !a)
                return dof::set_error(DOF_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            g_ptr[dev] = a;
        }
        ptr = g_ptr[dev];
    }
    return dof_render_frame(scene, cam, lens, gb, hist, p, out, ptr, kNoAllocScratchBytes, stream);
}
