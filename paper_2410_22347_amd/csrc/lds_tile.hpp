// Reads of a whole tile from the workgroup's LDS ring, one asm block per
// shape: every k-step block is requested, then one wait for all of them (the
// wait sits in the same block, so no load is in flight when the registers are
// handed back).  The outputs are early-clobber: a destination must never share
// a register with the address, which the later reads of the block still use
// while the earlier ones land.  lane_addr: LDS byte address of this lane's
// first element.
#pragma once

#include "search_common.hpp"

namespace gv {
namespace scan {

template <int KS, int EB8>  // EB8: bytes per lane per k-step (16: fp16/bf16, 8: fp8 in E4M3 bytes)
struct LdsTile;

template <>
struct LdsTile<2, 16> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[2], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b128 %0, %2 offset:0\n"
        "ds_read_b128 %1, %2 offset:1024\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<4, 16> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[4], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b128 %0, %4 offset:0\n"
        "ds_read_b128 %1, %4 offset:1024\n"
        "ds_read_b128 %2, %4 offset:2048\n"
        "ds_read_b128 %3, %4 offset:3072\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<8, 16> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[8], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b128 %0, %8 offset:0\n"
        "ds_read_b128 %1, %8 offset:1024\n"
        "ds_read_b128 %2, %8 offset:2048\n"
        "ds_read_b128 %3, %8 offset:3072\n"
        "ds_read_b128 %4, %8 offset:4096\n"
        "ds_read_b128 %5, %8 offset:5120\n"
        "ds_read_b128 %6, %8 offset:6144\n"
        "ds_read_b128 %7, %8 offset:7168\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]), "=&v"(d[7])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<10, 16> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[10], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b128 %0, %10 offset:0\n"
        "ds_read_b128 %1, %10 offset:1024\n"
        "ds_read_b128 %2, %10 offset:2048\n"
        "ds_read_b128 %3, %10 offset:3072\n"
        "ds_read_b128 %4, %10 offset:4096\n"
        "ds_read_b128 %5, %10 offset:5120\n"
        "ds_read_b128 %6, %10 offset:6144\n"
        "ds_read_b128 %7, %10 offset:7168\n"
        "ds_read_b128 %8, %10 offset:8192\n"
        "ds_read_b128 %9, %10 offset:9216\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]), "=&v"(d[7]), "=&v"(d[8]), "=&v"(d[9])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<12, 16> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[12], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b128 %0, %12 offset:0\n"
        "ds_read_b128 %1, %12 offset:1024\n"
        "ds_read_b128 %2, %12 offset:2048\n"
        "ds_read_b128 %3, %12 offset:3072\n"
        "ds_read_b128 %4, %12 offset:4096\n"
        "ds_read_b128 %5, %12 offset:5120\n"
        "ds_read_b128 %6, %12 offset:6144\n"
        "ds_read_b128 %7, %12 offset:7168\n"
        "ds_read_b128 %8, %12 offset:8192\n"
        "ds_read_b128 %9, %12 offset:9216\n"
        "ds_read_b128 %10, %12 offset:10240\n"
        "ds_read_b128 %11, %12 offset:11264\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]), "=&v"(d[7]), "=&v"(d[8]), "=&v"(d[9]), "=&v"(d[10]), "=&v"(d[11])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<16, 16> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[16], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b128 %0, %16 offset:0\n"
        "ds_read_b128 %1, %16 offset:1024\n"
        "ds_read_b128 %2, %16 offset:2048\n"
        "ds_read_b128 %3, %16 offset:3072\n"
        "ds_read_b128 %4, %16 offset:4096\n"
        "ds_read_b128 %5, %16 offset:5120\n"
        "ds_read_b128 %6, %16 offset:6144\n"
        "ds_read_b128 %7, %16 offset:7168\n"
        "ds_read_b128 %8, %16 offset:8192\n"
        "ds_read_b128 %9, %16 offset:9216\n"
        "ds_read_b128 %10, %16 offset:10240\n"
        "ds_read_b128 %11, %16 offset:11264\n"
        "ds_read_b128 %12, %16 offset:12288\n"
        "ds_read_b128 %13, %16 offset:13312\n"
        "ds_read_b128 %14, %16 offset:14336\n"
        "ds_read_b128 %15, %16 offset:15360\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]), "=&v"(d[7]), "=&v"(d[8]), "=&v"(d[9]), "=&v"(d[10]), "=&v"(d[11]), "=&v"(d[12]), "=&v"(d[13]), "=&v"(d[14]), "=&v"(d[15])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<2, 8> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[2], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b64 %0, %2 offset:0\n"
        "ds_read_b64 %1, %2 offset:512\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<4, 8> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[4], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b64 %0, %4 offset:0\n"
        "ds_read_b64 %1, %4 offset:512\n"
        "ds_read_b64 %2, %4 offset:1024\n"
        "ds_read_b64 %3, %4 offset:1536\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<8, 8> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[8], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b64 %0, %8 offset:0\n"
        "ds_read_b64 %1, %8 offset:512\n"
        "ds_read_b64 %2, %8 offset:1024\n"
        "ds_read_b64 %3, %8 offset:1536\n"
        "ds_read_b64 %4, %8 offset:2048\n"
        "ds_read_b64 %5, %8 offset:2560\n"
        "ds_read_b64 %6, %8 offset:3072\n"
        "ds_read_b64 %7, %8 offset:3584\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]), "=&v"(d[7])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<10, 8> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[10], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b64 %0, %10 offset:0\n"
        "ds_read_b64 %1, %10 offset:512\n"
        "ds_read_b64 %2, %10 offset:1024\n"
        "ds_read_b64 %3, %10 offset:1536\n"
        "ds_read_b64 %4, %10 offset:2048\n"
        "ds_read_b64 %5, %10 offset:2560\n"
        "ds_read_b64 %6, %10 offset:3072\n"
        "ds_read_b64 %7, %10 offset:3584\n"
        "ds_read_b64 %8, %10 offset:4096\n"
        "ds_read_b64 %9, %10 offset:4608\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]), "=&v"(d[7]), "=&v"(d[8]), "=&v"(d[9])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<12, 8> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[12], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b64 %0, %12 offset:0\n"
        "ds_read_b64 %1, %12 offset:512\n"
        "ds_read_b64 %2, %12 offset:1024\n"
        "ds_read_b64 %3, %12 offset:1536\n"
        "ds_read_b64 %4, %12 offset:2048\n"
        "ds_read_b64 %5, %12 offset:2560\n"
        "ds_read_b64 %6, %12 offset:3072\n"
        "ds_read_b64 %7, %12 offset:3584\n"
        "ds_read_b64 %8, %12 offset:4096\n"
        "ds_read_b64 %9, %12 offset:4608\n"
        "ds_read_b64 %10, %12 offset:5120\n"
        "ds_read_b64 %11, %12 offset:5632\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]), "=&v"(d[7]), "=&v"(d[8]), "=&v"(d[9]), "=&v"(d[10]), "=&v"(d[11])
        : "v"(lane_addr)
        : "memory");
  }
};

template <>
struct LdsTile<16, 8> {
  template <typename S>
  __device__ __forceinline__ static void read(S (&d)[16], uint32_t lane_addr) {
    asm volatile(
        "ds_read_b64 %0, %16 offset:0\n"
        "ds_read_b64 %1, %16 offset:512\n"
        "ds_read_b64 %2, %16 offset:1024\n"
        "ds_read_b64 %3, %16 offset:1536\n"
        "ds_read_b64 %4, %16 offset:2048\n"
        "ds_read_b64 %5, %16 offset:2560\n"
        "ds_read_b64 %6, %16 offset:3072\n"
        "ds_read_b64 %7, %16 offset:3584\n"
        "ds_read_b64 %8, %16 offset:4096\n"
        "ds_read_b64 %9, %16 offset:4608\n"
        "ds_read_b64 %10, %16 offset:5120\n"
        "ds_read_b64 %11, %16 offset:5632\n"
        "ds_read_b64 %12, %16 offset:6144\n"
        "ds_read_b64 %13, %16 offset:6656\n"
        "ds_read_b64 %14, %16 offset:7168\n"
        "ds_read_b64 %15, %16 offset:7680\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]), "=&v"(d[7]), "=&v"(d[8]), "=&v"(d[9]), "=&v"(d[10]), "=&v"(d[11]), "=&v"(d[12]), "=&v"(d[13]), "=&v"(d[14]), "=&v"(d[15])
        : "v"(lane_addr)
        : "memory");
  }
};

}  // namespace scan
}  // namespace gv
