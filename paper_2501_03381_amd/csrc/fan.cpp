// Fork/join of independent launches over per-device side streams (default priority).
//
// The register classes of one evaluation are independent grids of very different lengths; run on
// one stream, the short ones leave most compute units idle while the long ones drain.  A FanScope
// records an event on the caller's stream, makes up to kFanSide side streams wait for it, hands
// out the caller's stream and the side streams to the launches, and on destruction makes the
// caller's stream wait for every side stream it used.  Work before and after the scope on the
// caller's stream is therefore ordered exactly as with serial launches, and the pattern records
// into a HIP graph when the caller's stream is being captured (the side streams join the capture
// through the events).  Side streams are created on first use on a device, never while the
// caller's stream is capturing: such a first call runs its launches serially.  A mutex per process
// keeps the event records and waits of concurrent callers from interleaving.
#include "thoi_internal.hpp"

#include <cstdlib>
#include <mutex>

namespace thoi {
namespace {

constexpr int kMaxDevices = 64;

struct DevFan {
    bool tried = false, ok = false;
    hipStream_t side[kFanSide] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kFanSide] = {};
};

std::mutex g_mu;
DevFan g_dev[kMaxDevices];

bool fan_disabled()
{
    static const bool off = [] {
        const char* e = std::getenv("THOI_SERIAL_LAUNCH");
        return e && e[0] == '1';
    }();
    return off;
}

bool make_fan(DevFan& f, int dev)
{
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return false;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return false;
    bool ok = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < kFanSide; ++i) {
        ok = hipStreamCreateWithFlags(&f.side[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&f.join[i], hipEventDisableTiming) == hipSuccess;
    }
    if (cur != dev) (void)hipSetDevice(cur);
    return ok;
}

}  // namespace

FanScope::FanScope(hipStream_t s, int branches) : s_(s), lock_(g_mu, std::defer_lock)
{
    if (branches < 2 || fan_disabled()) return;
    int dev = 0;
    if (hipStreamGetDevice(s, &dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
    lock_.lock();
    DevFan& f = g_dev[dev];
    if (!f.tried) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
            lock_.unlock();
            return;                      // create the streams on a later, uncaptured call
        }
        f.tried = true;
        f.ok = make_fan(f, dev);
    }
    if (!f.ok || hipEventRecord(f.fork, s) != hipSuccess) {
        lock_.unlock();
        return;
    }
    fan_ = &f;
    nside_ = branches - 1 < kFanSide ? branches - 1 : kFanSide;
    for (int i = 0; i < nside_; ++i) {
        if (hipStreamWaitEvent(f.side[i], f.fork, 0) != hipSuccess) {
            nside_ = i;                  // launches beyond the streams that waited go to s
            break;
        }
    }
}

hipStream_t FanScope::stream(int branch) const
{
    if (!fan_ || branch <= 0) return s_;
    const int i = (branch - 1) % (nside_ + 1);
    return i < nside_ ? static_cast<DevFan*>(fan_)->side[i] : s_;
}

FanScope::~FanScope()
{
    if (!fan_) return;
    DevFan& f = *static_cast<DevFan*>(fan_);
    for (int i = 0; i < nside_; ++i) {
        if (hipEventRecord(f.join[i], f.side[i]) == hipSuccess) (void)hipStreamWaitEvent(s_, f.join[i], 0);
        else (void)hipStreamSynchronize(f.side[i]);      // cannot join on the device: join on the host
    }
    lock_.unlock();
}

}  // namespace thoi
