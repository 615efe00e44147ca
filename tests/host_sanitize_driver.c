/* Host-only calls of the library (bank, length classes, bank metric and
 * lattice placement), valid and invalid arguments, for a build with the
 * address and undefined-behaviour sanitizers on its host code.  Exits 0
 * when every call returns what its documentation states. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ci.h"

static int fails = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__,        \
              __LINE__, #cond);                                           \
      ++fails;                                                            \
    }                                                                     \
  } while (0)

/* a smooth coloured-noise PSD per Hz on the n/2 + 1 bins */
static double* make_psd(int64_t n, double fs) {
  double* s = (double*)malloc(sizeof(double) * (size_t)(n / 2 + 1));
  for (int64_t k = 0; k <= n / 2; ++k) {
    const double f = k == 0 ? fs / (double)n : (double)k * fs / (double)n;
    const double x = 150.0 / f;
    s[k] = 1e-46 * (x * x * x * x + 2.0 + 2.0 / (x * x));
  }
  return s;
}

int main(void) {
  /* bank */
  ci_template* bank = (ci_template*)malloc(sizeof(ci_template) * 1000);
  for (int kind = CI_BANK_GRID; kind <= CI_BANK_LOGUNIFORM; ++kind) {
    ci_bank_spec sp = {kind, 0, 1.0, 10.0, 42};
    EXPECT(ci_make_bank(&sp, 1000, bank) == CI_OK);
    for (int i = 0; i < 1000; ++i)
      EXPECT(bank[i].m1 >= bank[i].m2 && bank[i].m2 >= 1.0 && bank[i].m1 <= 10.0);
    EXPECT(ci_make_bank(&sp, 1, bank) == CI_OK);
    EXPECT(ci_make_bank(&sp, 0, NULL) == CI_OK);
  }
  {
    ci_bank_spec bad = {7, 0, 1.0, 10.0, 1};
    EXPECT(ci_make_bank(&bad, 10, bank) == CI_EINVAL);
    ci_bank_spec inv = {CI_BANK_UNIFORM, 0, 10.0, 1.0, 1};
    EXPECT(ci_make_bank(&inv, 10, bank) == CI_EINVAL);
    ci_bank_spec ok = {CI_BANK_UNIFORM, 0, 1.0, 10.0, 1};
    EXPECT(ci_make_bank(NULL, 10, bank) == CI_EINVAL);
    EXPECT(ci_make_bank(&ok, -1, bank) == CI_EINVAL);
    EXPECT(ci_make_bank(&ok, 10, NULL) == CI_EINVAL);
    EXPECT(ci_last_error(NULL) != NULL);
  }
  /* length classes */
  {
    const int64_t cls[4] = {1 << 17, 1 << 18, 1 << 19, 1 << 20};
    int32_t* out = (int32_t*)malloc(sizeof(int32_t) * 1000);
    EXPECT(ci_length_classes(bank, 1000, 4096.0, 20.0, cls, 4, out) == CI_OK);
    for (int i = 0; i < 1000; ++i) EXPECT(out[i] >= 0 && out[i] < 4);
    const int64_t unsorted[2] = {1 << 18, 1 << 17};
    EXPECT(ci_length_classes(bank, 1000, 4096.0, 20.0, unsorted, 2, out) == CI_EINVAL);
    EXPECT(ci_length_classes(bank, 1000, 4096.0, 20.0, cls, 0, out) == CI_EINVAL);
    free(out);
  }
  /* metric and lattice placement */
  {
    const int64_t n = 1 << 16;
    const double fs = 4096.0, fl = 30.0;
    double* psd = make_psd(n, fs);
    double g[3];
    EXPECT(ci_bank_metric(psd, n, fs, fl, 2.0, 1.5, g) == CI_OK);
    EXPECT(isfinite(g[0]) && g[0] > 0.0 && g[0] * g[2] - g[1] * g[1] > 0.0);
    EXPECT(ci_bank_metric(psd, n, fs, fl, -1.0, 1.5, g) == CI_EINVAL);
    EXPECT(ci_bank_metric(NULL, n, fs, fl, 2.0, 1.5, g) == CI_EINVAL);
    ci_lattice_spec ls = {3.0, 4.0, 0.97};
    int64_t count = -1;
    EXPECT(ci_make_bank_lattice(&ls, psd, n, fs, fl, NULL, 0, &count) == CI_OK);
    EXPECT(count > 0);
    if (count > 0) {
      ci_template* lat = (ci_template*)malloc(sizeof(ci_template) * (size_t)count);
      int64_t c2 = -1;
      EXPECT(ci_make_bank_lattice(&ls, psd, n, fs, fl, lat, count, &c2) == CI_OK);
      EXPECT(c2 == count);
      for (int64_t i = 0; i < c2; ++i)
        EXPECT(lat[i].m1 >= lat[i].m2 && lat[i].m2 >= 3.0 - 1e-9 && lat[i].m1 <= 4.0 + 1e-9);
      if (count > 1) {
        int64_t c3 = -1;
        EXPECT(ci_make_bank_lattice(&ls, psd, n, fs, fl, lat, count - 1, &c3) == CI_ETRUNC);
        EXPECT(c3 == count);
      }
      free(lat);
    }
    ci_lattice_spec bad = {4.0, 3.0, 0.97};
    EXPECT(ci_make_bank_lattice(&bad, psd, n, fs, fl, NULL, 0, &count) == CI_EINVAL);
    ci_lattice_spec badm = {3.0, 4.0, 1.5};
    EXPECT(ci_make_bank_lattice(&badm, psd, n, fs, fl, NULL, 0, &count) == CI_EINVAL);
    free(psd);
  }
  free(bank);
  if (fails) fprintf(stderr, "%d expectation(s) failed\n", fails);
  else printf("host calls ok\n");
  return fails ? 1 : 0;
}
