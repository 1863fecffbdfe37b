// Host-side helpers of the library (setup and launch wrappers).
#pragma once
#include <hip/hip_runtime.h>
#include <mutex>
#include <vector>

#include "mm_internal.h"

namespace mmh {
void demag_tensor(double X, double Y, double Z, double dx, double dy, double dz, double* out6);
int padded(int n);
void kernel_spectrum(int nx, int ny, int nz, double dx, double dy, double dz, std::vector<float>& out);
}  // namespace mmh

hipError_t mmk_launch_xfwd_cells(int method, int stage, int nblocks, const InstDesc* descs, const int* wg,
                                 const float2* tw, size_t lds, hipStream_t s);
hipError_t mmk_launch_stage(int method, int stage, bool final_pass, int nblocks, int count,
                            const InstDesc* descs, const int* wg, const float2* tw, size_t lds,
                            hipStream_t stream);
// x passes with lines in registers: Px = 4 MX, MX in {4, 8, 16, 32}; dir +1 forward (method,
// stage select the stage input), -1 inverse; work items are tiles of 128 rows
hipError_t mmk_launch_fft_xr(int dir, int MX, int nblocks, const InstDesc* d, const WorkItem* w, int method,
                             int stage, const float2* tw, hipStream_t s);
hipError_t mmk_launch_fft_xf(int W, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             int method, int stage, const float2* tw, hipStream_t s);
hipError_t mmk_launch_fft_xi(int W, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s);
// fused y-z with lines in registers: Py = 4 MY, Pz = 4 MZ, MY in {4,8,16,32}, MZ in {4,8,16}
hipError_t mmk_launch_fft_yzr(int MY, int MZ, int nblocks, size_t lds, const InstDesc* d,
                              const WorkItem* w, const float2* tw, hipStream_t s);
// the same with eight lanes per z column (512 threads): MY in {4,8,16,32}, MZ in {8,16}.
// nfinal > 0 appends that many workgroups that run the finalisation of stage
// fstage of method fmethod for instances 0 .. nfinal - 1.
hipError_t mmk_launch_fft_yz8(int MY, int MZ, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                              const float2* tw, hipStream_t s, int nfinal = 0, int fmethod = 0,
                              int fstage = 0);
hipError_t mmk_launch_fft_yzx(int MY, int MZ, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                              const float2* tw, hipStream_t s, int nfinal = 0, int fmethod = 0,
                              int fstage = 0);
int mmk_yzx_pad();
// k_fft_yzx for padded (py, pz) carries the real planes kx = 0 and Px/2 of an
// instance in one work item (item 0; no item Px/2), with 6 pz float2 more LDS
bool mmk_yzx_pairs(int py, int pz);
hipError_t mmk_launch_fft_ysx(int dir, int py, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                              const float2* tw, hipStream_t s, int nfinal = 0, int fmethod = 0,
                              int fstage = 0);
int mmk_sx_rows(int py);
hipError_t mmk_launch_fft_yz(int TK, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s);
hipError_t mmk_launch_fft_y(int dir, int W, int nblocks, size_t lds, const InstDesc* d,
                            const WorkItem* w, const float2* tw, hipStream_t s);
hipError_t mmk_launch_fft_zc(int TW, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s);
hipError_t mmk_set_lds_limits();
hipError_t mmk_launch_adj(int kind, int stage, int nblocks, int count, const InstDesc* d, const int* wg,
                          hipStream_t s, const float2* tw = nullptr, size_t lds = 0);
hipError_t mmk_launch_gather_done(int count, const InstDesc* d, int* out, hipStream_t s);
// the no-allocation run: this device's fixed scratch (address and size), the
// per-device lock that serialises such runs, and a zero-fill kernel
hipError_t mmk_noalloc_scratch(int dev, void** ptr, size_t* bytes);
std::mutex& mmk_noalloc_lock(int dev);
hipError_t mmk_launch_fill_zero(void* p, size_t bytes, hipStream_t s);
