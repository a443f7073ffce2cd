// tt_matvec_noalloc: the FP32 2RBT product of tt_matvec (§2.E) for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops).  Its kernels are those of tt_matvec; the transform work
// buffers that tt_matvec takes from the context (the row-pass output T and the
// column-pass output U, plus the projected input when low-order modes are
// removed) come from one file-scope device array instead, so the call itself
// allocates nothing.
//
// The array (`scratch`, SCRATCH_BYTES) lives on every device the library runs
// on until the process ends.  Its device address is looked up once per device
// with hipGetSymbolAddress when a context is created on that device (with the
// device current) and kept in scratch_ptr[device]; host code uses only that
// address, never the array's name.  Calls on one device share the array, so
// calls that overlap in time on one device (several streams or threads) race;
// every byte a call reads was written earlier by the same call (T by the row
// pass, U by the column pass, the projected input by its copy), so nothing
// needs clearing between calls.
#include "tt_internal.h"

#include <mutex>

namespace {

constexpr size_t SCRATCH_BYTES = size_t(8) << 20;    // 8 MiB per device
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES] = {};
hipError_t scratch_err[MAX_DEVICES] = {};
bool scratch_done[MAX_DEVICES] = {};

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

tt_status matvec_f32_into(tt_ctx& c, const float* x, float* y, c32* T, c32* U, float* tmp);

// Once per device, with that device current (called by tt_create).
void noalloc_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_done[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    scratch_err[device] = e;
    scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    scratch_done[device] = true;
}

size_t noalloc_scratch_bytes() { return SCRATCH_BYTES; }

tt_status tt_matvec_noalloc(tt_ctx* c, const float* d_x, float* d_y) {
    TT_REQUIRE(c && d_x && d_y, "NULL argument");
    TT_REQUIRE(d_x != d_y, "d_x and d_y must not alias");
    if (!c->ready) {
        tt_set_error("tt_matvec_noalloc: no system set");
        return TT_NOT_READY;
    }
    TT_REQUIRE(c->device >= 0 && c->device < MAX_DEVICES, "device index beyond the scratch table");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(scratch_mu);
        if (!scratch_done[c->device] || scratch_err[c->device] != hipSuccess || !scratch_ptr[c->device]) {
            tt_set_error(std::string("tt_matvec_noalloc: no scratch address for device ") +
                         std::to_string(c->device) + ": " +
                         (scratch_done[c->device] ? hipGetErrorString(scratch_err[c->device]) : "not looked up"));
            return TT_HIP_ERROR;
        }
        base = scratch_ptr[c->device];
    }
    const size_t tu = round256((size_t)c->Lh * c->C * c->n * sizeof(c32));
    const size_t tmp = c->modes ? round256((size_t)c->n_slopes * sizeof(float)) : 0;
    const size_t need = 2 * tu + tmp;
    if (need > SCRATCH_BYTES) {
        tt_set_error("tt_matvec_noalloc: the system needs " + std::to_string(need) +
                     " bytes of scratch (2 (pad_L/2 + 1) 2 n_gs n complex floats" +
                     (c->modes ? std::string(" + n_slopes floats") : std::string()) + "), above the " +
                     std::to_string(SCRATCH_BYTES) + "-byte limit; use tt_matvec");
        return TT_INVALID_ARG;
    }
    TT_HIP(hipSetDevice(c->device));
    unsigned char* b = static_cast<unsigned char*>(base);
    c32* T = reinterpret_cast<c32*>(b);
    c32* U = reinterpret_cast<c32*>(b + tu);
    float* t = c->modes ? reinterpret_cast<float*>(b + 2 * tu) : nullptr;
    return matvec_f32_into(*c, d_x, d_y, T, U, t);
}
