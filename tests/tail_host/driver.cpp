// Runs the library's coarse-tail kernel (the V-cycle below a level in one 1024-thread
// workgroup) on the CPU for a 2D FP64 hierarchy whose levels 1..4 are read from argv[1]:
// one host thread per work-item, workgroup barriers and wave shuffles emulated (shim.hpp);
// every buffer is a separate heap allocation of the size the library allocates, so
// AddressSanitizer reports any access outside them.  Prints the relative L2 difference of
// level 1's result from the reference in the same directory.
#include "adr_kernels_host.cpp"

using namespace adrk;
static std::vector<cx<double>> readc(const char *path, size_t n) {
  std::vector<cx<double>> v(n);
  FILE *f = fopen(path, "rb");
  if (!f || fread(v.data(), sizeof(cx<double>), n, f) != n) {
    printf("cannot read %s\n", path);
    exit(1);
  }
  fclose(f);
  return v;
}
template <typename T>
static T *heap_copy(const std::vector<T> &v) {
  T *p = new T[v.size()];
  std::copy(v.begin(), v.end(), p);
  return p;
}
int main(int argc, char **argv) {
  if (argc < 2) return 2;
  const char *dir = argv[1];
  constexpr int kMaxNu = 8;
  int nx[5], ny[5], N[5], nu[5];
  {
    char path[256];
    snprintf(path, sizeof path, "%s/meta.txt", dir);
    FILE *f = fopen(path, "r");
    for (int l = 1; l <= 4; ++l)
      if (fscanf(f, "%d %d %d %d", &nx[l], &ny[l], &N[l], &nu[l]) != 4) return 1;
    fclose(f);
  }
  TailArgs<double> A{};
  A.first = 1;
  A.last = 4;
  for (int l = 1; l <= 4; ++l) {
    TailLevel<double> &t = A.L[l];
    t.G.n[0] = nx[l];
    t.G.n[1] = ny[l];
    t.G.n[2] = 1;
    t.G.N = N[l];
    t.G.r0 = 1.0 / nx[l];
    t.G.r01 = 1.0 / ((double)nx[l] * ny[l]);
    char path[256];
    snprintf(path, sizeof path, "%s/planes%d.bin", dir, l);
    t.planes = heap_copy(readc(path, (size_t)21 * N[l]));
    snprintf(path, sizeof path, "%s/dinv%d.bin", dir, l);
    t.dinv = heap_copy(readc(path, N[l]));
    auto zeros = [&](size_t n) { return heap_copy(std::vector<cx<double>>(n, mk<double>(0.0, 0.0))); };
    t.x = zeros(N[l]);
    t.b = zeros(N[l]);
    t.r = zeros(N[l]);
    t.w = zeros(N[l]);
    t.V = zeros((size_t)N[l] * (kMaxNu + 1));
    t.Z = zeros((size_t)N[l] * (kMaxNu + 1));
    t.nu = nu[l];
  }
  {
    char path[256];
    snprintf(path, sizeof path, "%s/b1.bin", dir);
    auto b1 = readc(path, N[1]);
    std::copy(b1.begin(), b1.end(), A.L[1].b);
    snprintf(path, sizeof path, "%s/ainv.bin", dir);
    A.Ainv = heap_copy(readc(path, (size_t)N[4] * N[4]));
  }
  // The kernel argument lives in its own allocation, as the device copy does.
  TailArgs<double> *Ap = new TailArgs<double>(A);
  std::barrier<> block(1024);
  g_block_bar = &block;
  for (int w = 0; w < 16; ++w) g_wave_bar[w] = new std::barrier<>(64);
  std::vector<std::thread> th;
  th.reserve(1024);
  for (int t = 0; t < 1024; ++t)
    th.emplace_back([Ap, t] {
      threadIdx.x = t;
      k_coarse_tail<double, 2>(Ap);
    });
  for (auto &t : th) t.join();
  char path[256];
  snprintf(path, sizeof path, "%s/ref1.bin", dir);
  auto ref = readc(path, N[1]);
  double num = 0, den = 0;
  for (int i = 0; i < N[1]; ++i) {
    const double dr = A.L[1].x[i].re - ref[i].re, di = A.L[1].x[i].im - ref[i].im;
    num += dr * dr + di * di;
    den += ref[i].re * ref[i].re + ref[i].im * ref[i].im;
  }
  printf("rel_l2 %.6e\n", sqrt(num / den));
  return 0;
}
