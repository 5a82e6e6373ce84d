// Host-side check of the packed list entries (8-byte LINE2D and PLANE3D,
// one-word PLANE3D unit-weight): every value inside the
// limits round-trips exactly, every value outside is flagged.  Built with
// hipcc as host code (the entry functions are host-callable).
#include "../../paper_2107_11810_amd/csrc/gv_device.h"
#include <cstdio>
#include <cstdlib>

static int fails = 0;
#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);          \
      fails++;                                                         \
    }                                                                  \
  } while (0)

static LinS plane(int32_t K1, int32_t K2, int32_t F, int32_t w) {
  LinS s = lin_zero<FAM_PLANE3D>();
  s.K[0][0] = K1; s.K[0][1] = K2; s.F[0] = F; s.w = w;
  return s;
}
static LinS line(int32_t K, int32_t F, int32_t w) {
  LinS s = lin_zero<FAM_LINE2D>();
  s.K[0][0] = K; s.F[0] = F; s.w = w;
  return s;
}

int main() {
  static_assert(sizeof(EntP3p) == 8 && sizeof(EntL2p) == 8, "packed entries are 8 bytes");
  const int32_t ks[] = {0, 1, -1, 2, -2, 1000, -1000, GV_P3_KMAX, -GV_P3_KMAX, GV_P3_KMAX - 1, -GV_P3_KMAX + 1};
  const int32_t fs[] = {0, 1, -1, 12345, -12345, GV_P3_FMAX, -GV_P3_FMAX, GV_P3_FMAX - 1};
  const int32_t ws[] = {0, 1, 2, 63, 64, 65, 1000, 65535, 65536, GV_P3_WMAX, GV_P3_WMAX - 1};
  for (int32_t K1 : ks)
    for (int32_t K2 : ks)
      for (int32_t F : fs)
        for (int32_t w : ws) {
          bool ok = true;
          const EntP3p e = store_ent<FAM_PLANE3D, EntP3p>(plane(K1, K2, F, w), ok);
          const LinS r = load_ent<FAM_PLANE3D>(e);
          CHECK(ok);
          CHECK(r.K[0][0] == K1 && r.K[0][1] == K2 && r.F[0] == F && r.w == w);
        }
  // one field beyond its limit is flagged
  const LinS bad[] = {plane(GV_P3_KMAX + 1, 0, 0, 1), plane(0, -GV_P3_KMAX - 1, 0, 1), plane(0, 0, GV_P3_FMAX + 1, 1),
                      plane(0, 0, -GV_P3_FMAX - 1, 1), plane(0, 0, 0, GV_P3_WMAX + 1)};
  for (const LinS& s : bad) {
    bool ok = true;
    (void)store_ent<FAM_PLANE3D, EntP3p>(s, ok);
    CHECK(!ok);
  }
  // a flag once cleared stays cleared
  {
    bool ok = false;
    (void)store_ent<FAM_PLANE3D, EntP3p>(plane(0, 0, 0, 1), ok);
    CHECK(!ok);
  }
  // PLANE3D one-word unit-weight entry: 8-bit K1, K2, 16-bit F, weight 1
  static_assert(sizeof(EntP3u) == 4, "the one-word entry is 4 bytes");
  const int32_t ku[] = {0, 1, -1, 2, -2, 64, -64, 100, -100, GV_P3U_KMAX, -GV_P3U_KMAX, GV_P3U_KMAX - 1};
  for (int32_t K1 : ku)
    for (int32_t K2 : ku)
      for (int32_t F : fs) {
        bool ok = true;
        const EntP3u e = store_ent<FAM_PLANE3D, EntP3u>(plane(K1, K2, F, 1), ok);
        const LinS r = load_ent<FAM_PLANE3D>(e);
        CHECK(ok);
        CHECK(r.K[0][0] == K1 && r.K[0][1] == K2 && r.F[0] == F && r.w == 1);
      }
  const LinS badu[] = {plane(GV_P3U_KMAX + 1, 0, 0, 1), plane(0, -GV_P3U_KMAX - 1, 0, 1),
                       plane(0, 0, GV_P3_FMAX + 1, 1), plane(0, 0, -GV_P3_FMAX - 1, 1), plane(0, 0, 0, 2),
                       plane(0, 0, 0, 0)};
  for (const LinS& s : badu) {
    bool ok = true;
    (void)store_ent<FAM_PLANE3D, EntP3u>(s, ok);
    CHECK(!ok);
  }
  // LINE2D: 16-bit K and F, full 32-bit weight
  const int32_t ls[] = {0, 1, -1, 300, -300, GV_L2_MAX, -GV_L2_MAX};
  for (int32_t K : ls)
    for (int32_t F : ls)
      for (int32_t w : {1, 7, 100000, 2000000000}) {
        bool ok = true;
        const EntL2p e = store_ent<FAM_LINE2D, EntL2p>(line(K, F, w), ok);
        const LinS r = load_ent<FAM_LINE2D>(e);
        CHECK(ok);
        CHECK(r.K[0][0] == K && r.F[0] == F && r.w == w);
      }
  {
    bool ok = true;
    (void)store_ent<FAM_LINE2D, EntL2p>(line(GV_L2_MAX + 1, 0, 1), ok);
    CHECK(!ok);
  }
  {
    bool ok = true;
    (void)store_ent<FAM_LINE2D, EntL2p>(line(0, -GV_L2_MAX - 1, 1), ok);
    CHECK(!ok);
  }
  std::printf("%s\n", fails ? "FAILED" : "OK");
  return fails ? 1 : 0;
}
