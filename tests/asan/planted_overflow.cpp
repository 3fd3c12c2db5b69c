// A heap read one element past the end: the sanitizer build used for the ABI
// driver must report it (checks that the instrumentation is live).
#include <cstdio>
#include <vector>

int main(int argc, char**) {
  std::vector<double> v(8, 1.0);
  volatile double s = v.data()[7 + argc];
  std::printf("%f\n", (double)s);
  return 0;
}
