// CPU check of the host-side launch bounds (launch_checks.hpp): a split loop
// is launched only when its partial sums fit their buffer.
#include <cstdint>
#include <cstdio>

#include "../../paper_2601_04112_amd/csrc/launch_checks.hpp"

static int fails = 0;
static void expect(bool got, bool want, const char* what) {
  if (got != want) {
    std::printf("FAIL %s: got %d\n", what, (int)got);
    ++fails;
  }
}

int main() {
  using lsamg::split_fits;
  float buf[1];
  const void* p = buf;
  // exact fit and one over, for the 64-column buffers of a 9,021-row level
  expect(split_fits(16, 9021, 64, p, 16LL * 9021 * 64), true, "16 ranges fit exactly");
  expect(split_fits(17, 9021, 64, p, 16LL * 9021 * 64), false, "17 ranges overrun");
  expect(split_fits(4, 9021, 64, p, 4LL * 9021 * 64 - 1), false, "one scalar short");
  // a buffer sized for 16 columns, reused by a 64-column batch
  expect(split_fits(4, 113539, 64, p, 4LL * 113539 * 16), false, "16-column buffer, 64 columns");
  expect(split_fits(4, 113539, 16, p, 4LL * 113539 * 16), true, "16-column buffer, 16 columns");
  // no split: nothing is written, any buffer will do
  expect(split_fits(1, 1 << 30, 64, nullptr, 0), true, "no split");
  expect(split_fits(0, 5, 64, nullptr, 0), true, "split 0");
  // a split without a buffer, or with nonsense sizes
  expect(split_fits(2, 10, 64, nullptr, 1 << 20), false, "no buffer");
  expect(split_fits(2, -1, 64, p, 1 << 20), false, "negative rows");
  expect(split_fits(2, 10, 0, p, 1 << 20), false, "zero width");
  expect(split_fits(2, 0, 64, p, 1), true, "empty level");
  // products beyond 64 bits do not wrap around
  expect(split_fits(INT64_C(1) << 40, INT64_C(1) << 40, 64, p, INT64_MAX), false, "overflow");
  if (fails == 0) std::printf("launch checks ok\n");
  return fails == 0 ? 0 : 1;
}
