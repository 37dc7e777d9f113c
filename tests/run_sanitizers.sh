#!/bin/bash
# Host-side sanitizer run (CPU only; no GPU is touched): the oracle built with
# AddressSanitizer + UndefinedBehaviorSanitizer under its pin tests, and the
# HIP library's host code built with both under the C-ABI validation tests.
# Device code is not instrumented.  Writes its logs to $OUT (default /tmp/pp_san).
set -euo pipefail
ROOT=$(cd "$(dirname "$0")/.." && pwd)
OUT=${OUT:-/tmp/pp_san}
mkdir -p "$OUT"
cd "$ROOT"

gcc -O1 -g -std=c11 -fopenmp -fPIC -shared -fsanitize=address,undefined -fno-omit-frame-pointer \
    -o "$OUT/libpp_oracle_asan.so" oracle/pp_oracle.c -lm
PP_ORACLE_LIB="$OUT/libpp_oracle_asan.so" \
LD_PRELOAD="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)" \
ASAN_OPTIONS=detect_leaks=0:halt_on_error=1 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
    python -m pytest tests/test_oracle_pins.py tests/test_oracle_general.py -q -p no:cacheprovider \
    > "$OUT/oracle.log" 2>&1
tail -1 "$OUT/oracle.log"

for f in pp_kernels pp_fused pp_api; do
    /opt/rocm/bin/hipcc -O1 -g -std=c++17 --offload-arch=gfx950 -fPIC \
        -Xclang -target-feature -Xclang -packed-fp32-ops \
        -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
        -Xarch_host -fno-omit-frame-pointer \
        -I include -I paper_2012_11744_amd/csrc -c paper_2012_11744_amd/csrc/$f.hip -o "$OUT/$f.o"
done
/opt/rocm/bin/hipcc --offload-arch=gfx950 -shared -fPIC \
    -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
    -o "$OUT/libpp_asan.so" "$OUT/pp_kernels.o" "$OUT/pp_fused.o" "$OUT/pp_api.o"
ASANRT=$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -1)
PP_LIB="$OUT/libpp_asan.so" LD_PRELOAD="$ASANRT" \
ASAN_OPTIONS=detect_leaks=0:halt_on_error=1 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
    python -m pytest tests/test_abi.py -q -p no:cacheprovider > "$OUT/abi.log" 2>&1
tail -1 "$OUT/abi.log"
