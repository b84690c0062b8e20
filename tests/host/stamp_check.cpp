// Host check of the workspace stamps (wt_bin.hip: layout_stamp, count_stamp): a binned stream is accepted by a
// later call only under its own layout and record format, and a scatter only after a count of the same stream.
// Every pair of descriptions a caller could confuse must give different stamps; identical ones the same stamp.
#include <cstdio>
#include <vector>

#include "wt_bin.hip"

static unsigned long long lay(const wt_frame_desc& d, uint64_t frags, bool idx, size_t extra = 0) {
  const wt::Geom g = wt::make_geom(d, idx);
  const size_t bytes = wt::make_layout(g, frags).total + extra;
  return wt::layout_stamp(g, wt::make_layout(g, wt::capacity_for(g, bytes)), idx);
}

int main() {
  int bad = 0;
  auto expect = [&](bool ok, const char* what) {
    if (!ok) {
      printf("FAIL %s\n", what);
      ++bad;
    }
  };
  const wt_frame_desc base = {1920, 1080, 3, 1, WT_F32, 0};
  std::vector<std::pair<const char*, wt_frame_desc>> others = {
      {"rank 4", {1920, 1080, 4, 1, WT_F32, 0}},
      {"width 1919", {1919, 1080, 3, 1, WT_F32, 0}},
      {"height 1079", {1920, 1079, 3, 1, WT_F32, 0}},
      {"transposed", {1080, 1920, 3, 1, WT_F32, 0}},
      {"three channels", {1920, 1080, 3, 3, WT_F32, 0}},
      {"depth bounds", {1920, 1080, 3, 1, WT_F32, WT_TIGHT_DEPTH}},
      {"one pass", {1920, 1080, 3, 1, WT_F32, WT_TEMPORAL}},
      {"rank 2", {1920, 1080, 2, 1, WT_F32, 0}},
      {"4K", {3840, 2160, 3, 1, WT_F32, 0}},
  };
  const unsigned long long s0 = lay(base, 1000000, false);
  expect(s0 != 0, "stamp is never 0");
  expect(s0 == lay(base, 1000000, false), "same description, same stamp");
  // the coefficient storage type does not change the binning: a stream binned for FP32 serves FP16 storage
  wt_frame_desc f16 = base;
  f16.coeff_dtype = WT_F16;
  expect(s0 == lay(f16, 1000000, false), "storage type does not change the layout");
  for (auto& o : others) {
    const unsigned long long so = lay(o.second, 1000000, false);
    // a description whose geometry coincides exactly would be a valid reading of the same binned stream
    const wt::Geom ga = wt::make_geom(base), gb = wt::make_geom(o.second);
    const bool same_geom = ga.W == gb.W && ga.H == gb.H && ga.C == gb.C && ga.rank == gb.rank && ga.TW == gb.TW &&
                           ga.TH == gb.TH;
    if (!same_geom && so == s0) {
      printf("FAIL %s gives the stamp of the base description\n", o.first);
      ++bad;
    }
  }
  expect(lay(base, 1000000, false) != lay(base, 1000000, true), "gradient records differ from forward records");
  expect(lay(base, 1000000, false) != lay(base, 2000000, false), "another capacity is another layout");
  expect(lay(base, 1000000, false) != lay(base, 1000000, false, 4096), "another workspace size is another layout");
  // counts: the stream's size and addresses
  const wt::Geom g = wt::make_geom(base);
  const wt::Layout l = wt::make_layout(g, 1000000);
  const wt_fragments fa = {1000000, (const uint32_t*)0x1000, (const float*)0x2000, (const float*)0x3000,
                           (const float*)0x4000};
  wt_fragments fb = fa;
  const unsigned long long ca = wt::count_stamp(g, l, fa);
  expect(ca == wt::count_stamp(g, l, fb), "same stream, same count stamp");
  fb.count = 999999;
  expect(ca != wt::count_stamp(g, l, fb), "another count");
  fb = fa;
  fb.rgb = (const float*)0x5000;
  expect(ca != wt::count_stamp(g, l, fb), "another colour array");
  fb = fa;
  fb.pixel = (const uint32_t*)0x100001000ull;
  expect(ca != wt::count_stamp(g, l, fb), "another pixel array (high address bits)");
  expect(ca != wt::layout_stamp(g, l, false), "a count stamp is not a binning stamp");
  // the header the device fills
  expect(sizeof(wt::WsHeader) <= 256 && offsetof(wt::WsHeader, dropped) == 0, "header fits its 256 bytes");
  printf("stamps checked, bad %d\n", bad);
  return bad != 0;
}
