// ppc_host.hpp -- host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppc.h"

namespace ppc {

// Number of compute units of a device (cached; 256 on MI355X).
int device_cus(int device);

// Plain call on an explicit stream (argument checks included).
ppc_status plain_pospopcnt(unsigned width, uint64_t *counts, const void *buf, size_t nbytes, hipStream_t st);

// Plain call with positions relative to a stream start `offset` bytes
// before buf (width 0 = total popcount into counts[0]); optional events
// recorded by the first and last kernel dispatch.
ppc_status plain_pospopcnt_at(unsigned width, uint64_t *counts, const void *buf, size_t nbytes, uint64_t offset,
                              hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop);

// Launch geometry of the plain call on a device: the wave cap set with
// ppc_set_plain_geometry, else one 8-wave block on 3/4 of the CUs, and the
// waves per block.  Read once per call, so the pieces a long input is cut
// into and the grids that count them use the same pair.
struct PlainGeometry {
    unsigned waves;
    unsigned wpb;
};
PlainGeometry plain_geometry(int device);

// The same override, else one 8-wave block on every CU (the grid of the
// accumulation-schedule variants, whose extra ALU work wants every CU).
unsigned full_grid_wave_cap(int device);

}  // namespace ppc
