#!/usr/bin/env bash
# AddressSanitizer + UndefinedBehaviorSanitizer over the host code, on the CPU:
#  1. the FP64 oracle, built with -fsanitize=address,undefined, under the
#     CPU test suite (-m "not gpu");
#  2. the library's host side (argument checks, layouts, work lists) built
#     with the sanitizers on the host pass only, under the ABI tests, which
#     call every entry point's validation without a GPU.
# The sanitized builds go to a scratch folder and are loaded in place of the
# normal ones through ORACLE_LIB / SCPS_LIB; nothing in the tree is replaced.
# Usage: tests/run_sanitizers.sh   (exit status: that of the first failing step)
set -euo pipefail
ROOT="$(cd "$(dirname "$0")/.." && pwd)"
OUT="${SANITIZE_DIR:-/tmp/scps_sanitize}"
mkdir -p "$OUT"
export ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1"
export UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"

echo "== oracle (gcc, -fsanitize=address,undefined)"
gcc -O1 -g -std=c11 -fPIC -shared -fopenmp -fno-fast-math -fno-omit-frame-pointer \
    -fsanitize=address,undefined -fno-sanitize-recover=undefined \
    -o "$OUT/liboracle_san.so" "$ROOT/oracle/scps_oracle.c" -lm
(cd "$ROOT" && ORACLE_LIB="$OUT/liboracle_san.so" \
    LD_PRELOAD="$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so)" \
    timeout -k 10 600 python -m pytest tests -q -m "not gpu" -p no:cacheprovider)

echo "== library host side (hipcc, sanitizers on the host pass only)"
CLANG_RT="$(ls -d /opt/rocm/llvm/lib/clang/*/lib/linux | head -1)"
hipcc --offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -shared -munsafe-fp-atomics \
    -Xclang -target-feature -Xclang -packed-fp32-ops -fno-omit-frame-pointer \
    -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
    -Xarch_host -fno-sanitize-recover=undefined -shared-libsan \
    -I "$ROOT/include" -o "$OUT/libscps_san.so" \
    "$ROOT"/paper_1705_02180_amd/csrc/scps_kernels.hip "$ROOT"/paper_1705_02180_amd/csrc/scps_maps.hip \
    "$ROOT"/paper_1705_02180_amd/csrc/scps_funnel.hip "$ROOT"/paper_1705_02180_amd/csrc/scps_api.cpp
# clang's shared ASan runtime also carries the UBSan handlers (preloading the
# standalone UBSan runtime beside it deadlocks at start-up)
(cd "$ROOT" && SCPS_LIB="$OUT/libscps_san.so" LD_PRELOAD="$CLANG_RT/libclang_rt.asan-x86_64.so" \
    timeout -k 10 600 python -m pytest tests/test_abi.py -q -m "not gpu" -p no:cacheprovider)
echo "sanitizers: clean"
