/*
 * nn_device.h -- device-side generation inside HIP kernels (gfx950).
 *
 * Variates usually feed a simulation directly (Section 3.2), and Table 2
 * measures the generator with the memory traffic taken out.  This header
 * lets a consumer kernel make the sequence of Eq. 3 in registers, where the
 * variates are used, with no store to HBM.  Header-only; the host side
 * (nn.h) supplies the multipliers and the skip table:
 *
 *   host:    nn_dev_mult jump;  nn_dev_mult_pow(T, &jump);      // (2^53)^T
 *            const nn_dev_mult* tab;  nn_dev_skip_table(&tab);   // current device
 *   kernel:  double z = nn_dev_skip((double)state, t + 1, tab);  // element t + 1
 *            for (...) { double u = nn_dev_variate(z);  ...use u...;
 *                        z = nn_dev_mulmod(z, jump); }           // element t + 1 + T, ...
 *
 * reproduces, thread by thread, exactly the values nn_generate would store
 * at positions t, t + T, t + 2T, ... after `state`.  Compile the including
 * translation unit with -ffp-contract=off: the reduction depends on each
 * product being rounded on its own.
 *
 * A state is held as a double: an integer in [1, 3^33), exact in binary64.
 */
#ifndef NN_DEVICE_H
#define NN_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn.h"

/* v * z mod 3^33 for a state z and a multiplier m (nn_dev_mult_pow), exact.
 *
 * r = v z - q 3^33 with q = rint(z (qh + ql)), where qh + ql is v / 3^33 as
 * a double-double.  With m = 3^33 (2^52 < m < 2^53) and v, z in [1, m):
 *  - ph + pl == v z exactly (FMA two-product); v z < 2^105, so ph's ulp is
 *    at most 2^52 and |pl| <= 2^51;
 *  - |q - v z / m| <= 0.75 + 2^-52, because fl(z qh + fl(z ql)) is within
 *    one rounding of v z / m and rint adds at most 0.5 (0.5 in total once
 *    the estimate reaches 2^52, where its ulp is already 1); so r = v z - q m
 *    is an integer with |r| <= 0.76 m < 2^52;
 *  - t = fma(-q, m, ph) rounds the exact ph - q m = r - pl once; that is an
 *    integer of magnitude below 0.76 m + 2^51 < 2^53, so t is exact, and so
 *    is t + pl = r, an integer below 2^52;
 * so a single conditional add of m lands r in [1, m). */
__host__ __device__ __forceinline__ double nn_dev_mulmod(double z, nn_dev_mult m) {
    const double mod = 5559060566555523.0; /* 3^33 */
    const double ph = m.v * z;
    const double pl = __builtin_fma(m.v, z, -ph);
    const double e = __builtin_fma(z, m.qh, z * m.ql);
    const double q = __builtin_rint(e);
    const double r = __builtin_fma(-q, mod, ph) + pl;
    return r < 0.0 ? r + mod : r;
}

/* The variate of a state: RN(z * RN(3^-33)), as nn_generate's NN_OUT_F64. */
__host__ __device__ __forceinline__ double nn_dev_variate(double z) {
    return z * (1.0 / 5559060566555523.0);
}

/* The raw state as stored by nn_generate's NN_OUT_U64. */
__host__ __device__ __forceinline__ uint64_t nn_dev_state_bits(double z) {
    return (uint64_t)z;
}

/* One step of Eq. 3 with multiplier m: *z = m.v * *z mod 3^33, and returns
 * the new state's variate.  With m = nn_dev_mult_pow(1) this walks the
 * sequence element by element. */
__host__ __device__ __forceinline__ double nn_dev_next(double* z, nn_dev_mult m) {
    *z = nn_dev_mulmod(*z, m);
    return nn_dev_variate(*z);
}

/* z * (2^53)^k mod 3^33 for k < 2^56 (larger than the period) through the
 * library's skip table (nn_dev_skip_table: 7 levels of 256 entries, entry
 * [lvl][j] = (2^53)^(j * 256^lvl)); seven multiplications and seven table
 * reads, which a caller may first stage in LDS (42 KiB). */
__host__ __device__ __forceinline__ double nn_dev_skip(double z, uint64_t k,
                                                       const nn_dev_mult* table) {
    for (uint32_t lvl = 0; lvl < NN_DEV_SKIP_LEVELS; ++lvl)
        z = nn_dev_mulmod(z, table[lvl * NN_DEV_SKIP_SIZE + ((k >> (8 * lvl)) & 0xff)]);
    return z;
}

#endif /* NN_DEVICE_H */
