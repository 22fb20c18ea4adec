/* Bulk fills for the seeded input generator (same definition as the numpy
 * code in __init__.py: SplitMix64 output function at counter positions).
 * Holds no arithmetic of the method under test. */
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t base_of(uint64_t seed, uint64_t stream) { return mix64(seed * GAMMA + stream); }

/* out[i] = U01(seed, stream, start + i) */
void gfi_u01(uint64_t seed, uint64_t stream, uint64_t start, int64_t count, double *out)
{
    const uint64_t b = base_of(seed, stream);
    for (int64_t i = 0; i < count; ++i)
        out[i] = (double)(mix64(b + (start + (uint64_t)i + 1) * GAMMA) >> 11) * 0x1.0p-53;
}

/* n^3 grid (x fastest): interior U01 keyed by the linear index, zero boundary. */
void gfi_grid3d(int64_t n, uint64_t seed, uint64_t stream, double *u)
{
    const uint64_t b = base_of(seed, stream);
    for (int64_t z = 0; z < n; ++z)
        for (int64_t y = 0; y < n; ++y) {
            double *row = u + (z * n + y) * n;
            const int bnd_row = (z == 0 || z == n - 1 || y == 0 || y == n - 1);
            for (int64_t x = 0; x < n; ++x) {
                if (bnd_row || x == 0 || x == n - 1) {
                    row[x] = 0.0;
                } else {
                    const uint64_t idx = (uint64_t)((z * n + y) * n + x);
                    row[x] = (double)(mix64(b + (idx + 1) * GAMMA) >> 11) * 0x1.0p-53;
                }
            }
        }
}

/* keys[i] = (uint32)(H(seed, stream, start + i) >> 32) */
void gfi_keys_u32(uint64_t seed, uint64_t stream, uint64_t start, int64_t count, uint32_t *keys)
{
    const uint64_t b = base_of(seed, stream);
    for (int64_t i = 0; i < count; ++i)
        keys[i] = (uint32_t)(mix64(b + (start + (uint64_t)i + 1) * GAMMA) >> 32);
}

/* Zipf keys: rank index = smallest r with cdf[r] >= U01(seed, zstream, i)
 * (clamped to ranks-1), high 16 bits from H(seed, hstream, i) >> 48. */
void gfi_keys_zipf(uint64_t seed, uint64_t zstream, uint64_t hstream, int64_t count, const double *cdf,
                   int64_t ranks, uint32_t *keys)
{
    const uint64_t bz = base_of(seed, zstream), bh = base_of(seed, hstream);
    for (int64_t i = 0; i < count; ++i) {
        const double u = (double)(mix64(bz + ((uint64_t)i + 1) * GAMMA) >> 11) * 0x1.0p-53;
        int64_t lo = 0, hi = ranks; /* first index in [lo, hi) with cdf >= u */
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] < u)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo > ranks - 1)
            lo = ranks - 1;
        const uint32_t hi16 = (uint32_t)(mix64(bh + ((uint64_t)i + 1) * GAMMA) >> 48);
        keys[i] = (uint32_t)lo | (hi16 << 16);
    }
}
