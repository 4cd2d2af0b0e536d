// Third, independent Philox4x32-10: rocRAND's open-source engine, run on the
// host.  Reads n records of (counter[4], key[2]) uint32 from argv[1], writes
// the n output blocks (4 x uint32) to argv[2].  Used only by the test-suite.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>
#include <cstdio>
#include <vector>

int main(int argc, char** argv)
{
    if (argc != 3) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    std::vector<uint32_t> in;
    uint32_t rec[6];
    while (std::fread(rec, sizeof(uint32_t), 6, f) == 6) in.insert(in.end(), rec, rec + 6);
    std::fclose(f);
    size_t n = in.size() / 6;
    std::vector<uint32_t> out(4 * n);
    for (size_t i = 0; i < n; ++i) {
        const uint32_t* r = &in[6 * i];
        unsigned long long seed = (unsigned long long)r[4] | ((unsigned long long)r[5] << 32);
        unsigned long long sub = (unsigned long long)r[2] | ((unsigned long long)r[3] << 32);
        unsigned long long off = ((unsigned long long)r[0] | ((unsigned long long)r[1] << 32)) * 4ull;
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        for (int k = 0; k < 4; ++k) out[4 * i + k] = e();
    }
    FILE* g = std::fopen(argv[2], "wb");
    if (!g) return 4;
    std::fwrite(out.data(), sizeof(uint32_t), out.size(), g);
    std::fclose(g);
    return 0;
}
