// Host-side launchers of the grouped kernels (defined next to the kernels).
#pragma once
#include <hip/hip_runtime.h>
#include "jobs.hpp"
#include "small.hpp"

namespace rg {

void launch_zero(void* p, int64_t bytes, hipStream_t st);
void launch_zerog(const ZeroJob* j, const int* pre, int nj, int tiles, hipStream_t st);
void launch_gen(bool f64, const GenJob* j, const int* pre, int nj, int tiles, hipStream_t st);
void launch_ab(int prec, int ta, int tb, int td, int ct, int js, const AbJob* j, const int* pre,
               int nj, int tiles, hipStream_t st);
void launch_gram(int tx, int rgs, const GramJob* j, const int* pre, int nj, int tiles, hipStream_t st);
void launch_reduce(int ti, int to, bool sym, const RedJob* j, const int* pre, int nj, int tiles,
                   hipStream_t st);
void launch_chol(const CholJob* j, int nj, hipStream_t st);
void launch_small(const SmallJob* j, int nj, hipStream_t st);
void launch_bjinit(const BJJob* j, int nj, int sweep, hipStream_t st);
void launch_bjround(const BJJob* j, const int* pre, int nj, int tiles, int sweep, int round, hipStream_t st);
void launch_bjsweep(const BJJob* j, const int* pre, int nj, int tiles, int sweep, int sw0, int spin,
                    hipStream_t st);
void launch_sign(const SignJob* j, const int* pre, int nj, int tiles, hipStream_t st);
void launch_scale(const SignJob* j, const int* pre, int nj, int tiles, hipStream_t st);

}  // namespace rg

namespace rg {
void launch_gw(int prec, int gdt, int rt, int ct, const NnJob* j, const int* pre, int nj, int tiles,
               hipStream_t st);
// FP32 G, FP32 pass, packed W: 4-wave workgroups of 64 rows
void launch_gw4(int prec, int ct, const NnJob* j, const int* pre, int nj, int tiles, hipStream_t st);
void launch_nn(bool split, int rt, int ct, const NnJob* j, const int* pre, int nj, int tiles, hipStream_t st);
void launch_gtq(int prec, int gdt, int ct, int js, const AbJob* j, const int* pre, int nj, int tiles,
                hipStream_t st);
// waves per workgroup of k_tn; each wave covers 32 columns of G
constexpr int TN_WAVES = 8;
void launch_tn(bool split, int ct, const AbJob* j, const int* pre, int nj, int tiles, hipStream_t st);
int tn_tiles_per_chunk(bool split, int ct, int n);
void launch_pack(const void* j, const int* pre, int nj, int tiles, hipStream_t st);
}  // namespace rg
