// ap_nblist_build_noalloc: the neighbour-list build of ap_nblist_build without a context and without any
// allocation. Its scratch (wrapped positions, cell arrays, the cells' records, flags) lives in one
// file-scope device array per GPU, sized for at most kNoAllocMaxAtoms atoms and kNoAllocMaxCells cells.
#include <cstring>
#include <mutex>

#include "ap_internal.h"

namespace ap {

constexpr int kNoAllocMaxAtoms = 1 << 17;
constexpr int kNoAllocMaxCells = 1 << 17;
constexpr int kNoAllocMaxDevices = 64;

// byte offsets of the pieces (each a multiple of 256)
constexpr size_t kRound = 256;
constexpr size_t rnd(size_t b) { return (b + kRound - 1) / kRound * kRound; }
constexpr size_t kOffRec = 0;
constexpr size_t kOffPos = kOffRec + rnd(sizeof(CandRec) * kNoAllocMaxAtoms);
constexpr size_t kOffPosBuild = kOffPos + rnd(3 * sizeof(double) * kNoAllocMaxAtoms);
constexpr size_t kOffCellOf = kOffPosBuild + rnd(3 * sizeof(double) * kNoAllocMaxAtoms);
constexpr size_t kOffCellAtoms = kOffCellOf + rnd(sizeof(int) * kNoAllocMaxAtoms);
constexpr size_t kOffShort = kOffCellAtoms + rnd(sizeof(int) * kNoAllocMaxAtoms);
constexpr size_t kOffCnt = kOffShort + rnd(sizeof(int) * kNoAllocMaxAtoms);
constexpr size_t kOffStart = kOffCnt + rnd(sizeof(int) * kNoAllocMaxCells);
constexpr size_t kOffFill = kOffStart + rnd(sizeof(int) * (kNoAllocMaxCells + 1));
constexpr size_t kOffFlags = kOffFill + rnd(sizeof(int) * kNoAllocMaxCells);
constexpr size_t kScratchBytes = kOffFlags + rnd(sizeof(int) * 8);  // 11.0 MiB

// One copy per GPU, held until the process ends. Host code never passes this name to a kernel (on the
// host it is only a stand-in); it uses the device address looked up per device below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kNoAllocMaxDevices];

// The device address of this GPU's scratch array, looked up once per device with the device current.
static int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error_text(AP_E_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kNoAllocMaxDevices) return set_error_text(AP_E_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return set_error_text(AP_E_HIP, "hipGetSymbolAddress(scratch) failed");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AP_OK;
}

}  // namespace ap

using namespace ap;

extern "C" int ap_nblist_build_noalloc(int n, const double *pos, const ap_box *box, double r_list, int max_nbr,
                                       int32_t *nbr_count, int32_t *nbr_idx, void *hip_stream) {
    if (n <= 0 || !pos || !box || !nbr_count || !nbr_idx || !(r_list > 0) || max_nbr <= 0 || max_nbr > 1536)
        return set_error_text(AP_E_ARG, "n > 0, pos, box, r_list > 0, 0 < max_nbr <= 1536 and outputs required");
    if (n > kNoAllocMaxAtoms) return set_error_text(AP_E_ARG, "n above the scratch limit of 131072 atoms");
    for (int a = 0; a < 3; a++)
        if (!(box->L[a] > 0) || !std::isfinite(box->L[a])) return set_error_text(AP_E_ARG, "box lengths must be > 0");
    Geometry g;
    if (!list_geometry(box->L, r_list, g))
        return set_error_text(AP_E_BOX, "list radius must be below half the box");
    if (g.ncell > kNoAllocMaxCells) return set_error_text(AP_E_ARG, "more cells than the scratch limit of 131072");
    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    unsigned char *sb = static_cast<unsigned char *>(base);
    hipStream_t s = (hipStream_t)hip_stream;
    double *wpos = reinterpret_cast<double *>(sb + kOffPos);
    int *flags = reinterpret_cast<int *>(sb + kOffFlags);
    int *cell_cnt = reinterpret_cast<int *>(sb + kOffCnt);
    int *cell_fill = reinterpret_cast<int *>(sb + kOffFill);
    const ListBufs b{wpos,
                     reinterpret_cast<double *>(sb + kOffPosBuild),
                     flags,
                     reinterpret_cast<int *>(sb + kOffCellOf),
                     cell_cnt,
                     reinterpret_cast<int *>(sb + kOffStart),
                     cell_fill,
                     reinterpret_cast<int *>(sb + kOffCellAtoms),
                     reinterpret_cast<CandRec *>(sb + kOffRec),
                     nbr_count,
                     reinterpret_cast<int32_t *>(sb + kOffShort),
                     nbr_idx};
    // the array keeps the previous call's contents: the build flag, the error bits and the cell counters
    // start from fill kernels (no memset nodes), every other piece is written before it is read
    launch_fill_int_on(s, flags, 0, 8);
    launch_fill_int_on(s, flags, 1, 1);
    launch_fill_int_on(s, cell_cnt, 0, g.ncell);
    launch_fill_int_on(s, cell_fill, 0, g.ncell);
    launch_wrap(s, pos, wpos, n, box->L);
    // every hit in the front part of the slots, in scan order (no short partition without a potential)
    launch_list_kernels(s, n, g, r_list, r_list, max_nbr, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error_text(AP_E_HIP, "list kernels failed to launch");
    int host_flags[2] = {0, 0};
    e = hipMemcpyAsync(host_flags, flags, sizeof(host_flags), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error_text(AP_E_HIP, "stream synchronize failed");
    if (host_flags[1] & kErrOverflow) return set_error_text(AP_E_NBR_OVERFLOW, "neighbour count above max_nbr");
    return AP_OK;
}
