// Sliced ELLPACK: host builder and device copies.
#include "sell.hpp"

#include <algorithm>

namespace pfx {

namespace {
constexpr int SLICE = 64;
}  // namespace

// Rows (a multiple of 64 of them) into slices of 64 consecutive rows.  Each
// slice's width is at least 1 and a multiple of `quantum` (padding entries are
// zeros), so that kernels may read a slice's last entry unconditionally and
// unroll by the quantum without a remainder.
SellHost build_sell(const std::vector<SellRow>& rows, int quantum) {
  SellHost h;
  const int ns = (int)rows.size() / SLICE;
  h.off.resize(ns);
  h.width.resize(ns);
  int cur = 0;
  for (int s = 0; s < ns; ++s) {
    int w = 1;
    for (int l = 0; l < SLICE; ++l) w = std::max(w, (int)rows[s * SLICE + l].size());
    w = (w + quantum - 1) / quantum * quantum;
    h.off[s] = cur;
    h.width[s] = w;
    cur += SLICE * w;
  }
  h.col.assign(cur, 0);
  h.re.assign(cur, 0.0);
  h.im.assign(cur, 0.0);
  for (int s = 0; s < ns; ++s)
    for (int l = 0; l < SLICE; ++l) {
      const SellRow& r = rows[s * SLICE + l];
      for (size_t p = 0; p < r.size(); ++p) {
        const int q = h.off[s] + (int)p * SLICE + l;
        h.col[q] = std::get<0>(r[p]);
        h.re[q] = std::get<1>(r[p]);
        h.im[q] = std::get<2>(r[p]);
      }
      h.entries += (long)r.size();
    }
  return h;
}

void upload_sell(Context* ctx, const SellHost& h, bool cplx, SellBuffers& b) {
  b.n_slices = (int)h.off.size();
  b.entries = h.entries;
  b.off = upload(ctx, h.off);
  b.width = upload(ctx, h.width);
  b.col = upload(ctx, h.col);
  if (cplx) {
    std::vector<double> v64(2 * h.re.size());
    std::vector<float> v32(2 * h.re.size());
    for (size_t i = 0; i < h.re.size(); ++i) {
      v64[2 * i] = h.re[i];
      v64[2 * i + 1] = h.im[i];
      v32[2 * i] = (float)h.re[i];
      v32[2 * i + 1] = (float)h.im[i];
    }
    b.val64 = upload(ctx, v64);
    b.val32 = upload(ctx, v32);
  } else {
    b.val64 = upload(ctx, h.re);
    b.val32 = upload(ctx, std::vector<float>(h.re.begin(), h.re.end()));
  }
}

std::pair<std::vector<int>, std::vector<int>> upload_psell(Context* ctx, const std::vector<SellRow>& rows,
                                                           PSellBuffers& b, bool cplx) {
  const int ns = (int)rows.size() / SLICE;
  std::vector<int> off(ns), width(ns);
  int cur = 0;
  for (int s = 0; s < ns; ++s) {
    int w = 1;
    for (int l = 0; l < SLICE; ++l) w = std::max(w, (int)rows[s * SLICE + l].size());
    off[s] = cur;
    width[s] = (w + 3) / 4;
    cur += SLICE * width[s];
  }
  std::vector<unsigned short> col((size_t)4 * cur, 0);
  std::vector<double> val((size_t)4 * cur, 0.0), vim(cplx ? (size_t)4 * cur : 0, 0.0);
  long entries = 0;
  for (int s = 0; s < ns; ++s)
    for (int l = 0; l < SLICE; ++l) {
      const SellRow& r = rows[s * SLICE + l];
      for (size_t p = 0; p < r.size(); ++p) {
        const int c = std::get<0>(r[p]);
        if (c < 0 || c > 65535) fail(PF_INVALID_ARG, "packed layout needs columns below 65536");
        const size_t q = 4 * ((size_t)off[s] + (p / 4) * SLICE + l) + p % 4;
        col[q] = (unsigned short)c;
        val[q] = std::get<1>(r[p]);
        if (cplx) vim[q] = std::get<2>(r[p]);
      }
      entries += (long)r.size();
    }
  b.n_slices = ns;
  b.entries = entries;
  b.off = upload(ctx, off);
  b.width = upload(ctx, width);
  b.col = upload(ctx, col);
  if (cplx) {
    std::vector<double> v64(2 * val.size());
    std::vector<float> v32(2 * val.size());
    for (size_t i = 0; i < val.size(); ++i) {
      v64[2 * i] = val[i];
      v64[2 * i + 1] = vim[i];
      v32[2 * i] = (float)val[i];
      v32[2 * i + 1] = (float)vim[i];
    }
    b.val64 = upload(ctx, v64);
    b.val32 = upload(ctx, v32);
  } else {
    b.val64 = upload(ctx, val);
    b.val32 = upload(ctx, std::vector<float>(val.begin(), val.end()));
  }
  return {off, width};
}

template <>
PSell<double> PSellBuffers::view<double>() const {
  return PSell<double>{off.as<int>(), width.as<int>(), col.as<unsigned short>(), val64.as<double>()};
}
template <>
PSell<float> PSellBuffers::view<float>() const {
  return PSell<float>{off.as<int>(), width.as<int>(), col.as<unsigned short>(), val32.as<float>()};
}

template <>
PSell<double2> PSellBuffers::view<double2>() const {
  return PSell<double2>{off.as<int>(), width.as<int>(), col.as<unsigned short>(), val64.as<double2>()};
}
template <>
PSell<float2> PSellBuffers::view<float2>() const {
  return PSell<float2>{off.as<int>(), width.as<int>(), col.as<unsigned short>(), val32.as<float2>()};
}

template <>
Sell<double> SellBuffers::view<double>() const {
  return Sell<double>{off.as<int>(), width.as<int>(), col.as<int>(), val64.as<double>()};
}
template <>
Sell<float> SellBuffers::view<float>() const {
  return Sell<float>{off.as<int>(), width.as<int>(), col.as<int>(), val32.as<float>()};
}
template <>
Sell<double2> SellBuffers::view<double2>() const {
  return Sell<double2>{off.as<int>(), width.as<int>(), col.as<int>(), val64.as<double2>()};
}
template <>
Sell<float2> SellBuffers::view<float2>() const {
  return Sell<float2>{off.as<int>(), width.as<int>(), col.as<int>(), val32.as<float2>()};
}

}  // namespace pfx
