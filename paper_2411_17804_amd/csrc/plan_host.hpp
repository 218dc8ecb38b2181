// plan_host.hpp -- the host side of the library that needs no GPU: argument
// validation and the FP64 plan builder (per station and channel: nearest
// cells, separable kernel weights, the gather lists cell -> taps).  Nothing
// here includes device code, so it also builds with a plain host compiler
// (the sanitizer build of the tests).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "epic.h"

namespace epic {

// One kernel tap of the gather: the element and its FP32 weight.
struct Tap {
    int32_t elem;
    float w;
};

// Footprint box of one (station, channel) and its entries in the tables.
struct ChanPlan {
    int32_t x0, y0, bw, bh;   // footprint box of this channel
    int64_t cell_off;         // first entry of this channel in cell_start[]
    int64_t tap_off;          // first entry of this channel in taps[]
    float wsum_max;           // max over cells of the sum of |weight| of its taps
    int32_t pad_;
};

// The plan of one station on the host (FP64 computed, FP32 stored).  Per
// channel c: chans[c] and, from chans[c].cell_off, cell_start[bw*bh + 1]
// (tap offsets relative to tap_off), then the box cells by descending tap
// count and a -1 (cell_order, same offsets); from tap_off, the taps in cell
// order, ascending element order within a cell.  elem_cell[c][a] is element
// a's nearest cell ci | cj << 16.
//
// Stations of at least kBandMinElem elements also get the tables of the
// row-band gather: per channel each element's slot in the order of the
// elements' nearest-cell rows (stable in element order: band_slot[c][e]), the
// first slot of each grid row (band_row[c][y], y = 0 .. ny), and a copy of
// the taps with each element replaced by its slot (band_taps, same offsets as
// taps).
// The elements whose footprints reach row y are then the slots
// [band_row[y - h], band_row[y + h + 1]) (h = half the kernel support), at most
// max_band of them.
constexpr int kBandMinElem = 8192;

struct HostPlan {
    std::vector<ChanPlan> chans;
    std::vector<int32_t> cell_start;
    std::vector<int32_t> cell_order;
    std::vector<int32_t> elem_cell;
    std::vector<Tap> taps;
    std::vector<int32_t> band_slot;
    std::vector<int32_t> band_row;
    std::vector<Tap> band_taps;
    int32_t max_box = 0, max_bw = 0, max_bh = 0, max_cell_taps = 0;
    int32_t max_band = 0;       // 0: no row-band tables
};

// Error detail of the calling thread (epic_last_error).
void set_error(const std::string &msg);
epic_status fail(epic_status st, const std::string &msg);
const char *last_error_cstr();

bool is_pow2_grid(int n);
epic_status check_common(const epic_common *c);
epic_status check_station(const epic_station *s, int idx, bool need_volts = true);

// Nearest cell and separable weights of one element at one channel (grid
// spacing delta metres); false if the footprint leaves the grid.
bool element_taps(double x, double y, double delta, int nx, int ny, const epic_kernel &kn, int *ci,
                  int *cj, double *wx, double *wy);

// Every element's footprint stays on the grid at every channel.
epic_status check_geometry(const epic_common *common, const epic_station *st);

// The plan tables of one station (validates the geometry first).
epic_status build_host_plan(const epic_common *common, const epic_station *st, HostPlan *out);

}  // namespace epic
