// layout.hpp -- row pitch of the half-spectrum buffers, shared by the host
// allocation and the device bodies.
#pragma once

namespace mmk {

// A row of the half spectrum holds nx + 1 complex values (kx = 0..nx).  Rows
// start on 64-byte boundaries (a pitch of a multiple of 8 complex values):
// a workgroup tile of 8 (16, 32) kx columns then touches exactly one (two,
// four) 64-byte segments per row instead of straddling two (three, five).
// K~ rows use the same pitch, with six floats per frequency.
__host__ __device__ constexpr int x_pitch(int nxc) { return (nxc + 7) & ~7; }

}  // namespace mmk
