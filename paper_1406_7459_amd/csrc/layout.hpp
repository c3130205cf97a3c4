// layout.hpp -- row pitch of the half-spectrum buffers and the workgroup to
// XCD mapping, shared by the host allocation and the device code.
#pragma once
#include <hip/hip_runtime.h>

namespace mmk {

// A row of the half spectrum holds nx + 1 complex values (kx = 0..nx).  Rows
// start on 128-byte boundaries (a pitch of a multiple of 16 complex values),
// the size of every read request the L2 sends to HBM: a tile of 16 kx
// columns then reads whole 128-byte lines, and narrower tiles share lines
// only with their neighbours in the same row.  K~ rows use the same pitch,
// with six floats per frequency.
__host__ __device__ constexpr int x_pitch(int nxc) { return (nxc + 15) & ~15; }

// Workgroups are dealt to the 8 XCDs round-robin in launch order, and each
// XCD has its own L2.  This maps launch id b (of nb) to a logical id so that
// XCD x runs the contiguous logical range [x nb/8, (x+1) nb/8) in order:
// logical neighbours (tiles sharing 128-byte lines, mirror rows sharing a K~
// row, neighbour cell planes) meet in one L2 at nearly the same time.  Ids
// past the last multiple of 8 keep their place.
// Stride between the (component, z) planes of the y-transformed spectrum
// X2, in complex elements: Ly rows of xp plus 128 bytes.  Without the pad
// the z pass's rows of one column sit a multiple of 16 KiB apart (256 rows
// of 1088 bytes at Ly = 256), so one workgroup's loads share their low
// address bits and crowd into few HBM channels.
__host__ __device__ constexpr int x2_plane_stride(int Ly, int xp) { return Ly * xp + 16; }

__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned per = nb / 8u;
    if (per == 0u || b >= per * 8u) return b;
    return (b % 8u) * per + b / 8u;
}

}  // namespace mmk
