// Sliced ELLPACK (SELL) storage shared by the solvers: device view, host
// builder and device copies.
#pragma once

#include <hip/hip_runtime.h>

#include <tuple>
#include <utility>
#include <vector>

#include "common.hpp"

namespace pfx {

// Sliced ELLPACK: rows are grouped in slices of 64 (one wavefront), each
// slice padded to its longest row.  Entry p of the row on lane l of slice s
// sits at off[s] + 64 p + l; padding entries have column 0 and value 0.
template <typename V>
struct Sell {
  const int* off;     // [n_slices]
  const int* width;   // [n_slices]
  const int* col;
  const V* val;
};

// Packed sliced layout: the slices of Sell, but each lane's entries are
// grouped in fours.  Group g of the row on lane l of slice s is group index
// off[s] + 64 g + l; it holds four values (val[4 index ..]) and four 16-bit
// columns (col[4 index ..]), so a group is one 8-byte column load and
// sizeof(V) / 4 16-byte value loads.  Offsets and widths count groups;
// padding entries have column 0 and value 0.  Entry p of that row is entry
// 4 (off[s] + 64 (p / 4) + l) + p % 4 of the value array.
template <typename V>
struct PSell {
  const int* off;
  const int* width;
  const unsigned short* col;
  const V* val;
};

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

// Host-built sliced ELLPACK with device copies of its values in FP64 and FP32.
struct SellBuffers {
  int n_slices = 0;
  long entries = 0;
  DeviceBuffer off, width, col, val64, val32;
  template <typename V>
  Sell<V> view() const;
};

// Host side: rows (a multiple of 64 of them) as (column, value re, value im)
// lists; builds slices of 64 consecutive rows whose widths are at least 1 and
// multiples of `quantum` (padding entries are zeros).
using SellEntry = std::tuple<int, double, double>;
using SellRow = std::vector<SellEntry>;

struct SellHost {
  std::vector<int> off, width, col;
  std::vector<double> re, im;
  long entries = 0;
};

SellHost build_sell(const std::vector<SellRow>& rows, int quantum = 1);

// Device copies: values in FP64 and FP32, complex values as (re, im) pairs.
void upload_sell(Context* ctx, const SellHost& h, bool cplx, SellBuffers& b);

// Packed layout (columns below 65536) with device copies of its values in
// FP64 and FP32 (complex values as (re, im) pairs); rows as for build_sell (a
// multiple of 64).
struct PSellBuffers {
  int n_slices = 0;
  long entries = 0;
  DeviceBuffer off, width, col, val64, val32;
  template <typename V>
  PSell<V> view() const;
};
// Returns the slices' group offsets and widths (as uploaded).
std::pair<std::vector<int>, std::vector<int>> upload_psell(Context* ctx, const std::vector<SellRow>& rows,
                                                           PSellBuffers& b, bool cplx = false);

}  // namespace pfx
