// A deliberate data race in an OpenMP loop: built and run like the host code
// under ThreadSanitizer, it must be reported, so that a clean run of the host
// code means something (the race detector and the OpenMP annotations work).
#include <cstdio>

int main() {
    long sum = 0;
#pragma omp parallel for
    for (int i = 0; i < 200000; ++i) sum += i;  // unsynchronised read-modify-write: a race
    std::printf("%ld\n", sum);
    return 0;
}
