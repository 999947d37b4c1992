#!/bin/bash
# The CPU test suite (-m "not gpu") under AddressSanitizer and
# UndefinedBehaviorSanitizer: the host code of the HIP library (argument
# validation, workspace and descriptor arithmetic, tuner cache parsing,
# solver and scheduler bookkeeping) and the C oracle, both instrumented and
# built with clang so that one sanitizer runtime serves them; that runtime
# is preloaded into the (uninstrumented) Python interpreter.  Leak detection
# is off: the interpreter's own allocations would be reported at exit.
# Usage: tests/sanitize.sh [extra pytest args]
set -euo pipefail
cd "$(dirname "$0")/.."
python -m paper_0911_3191_amd.build --sanitize
python -c 'import oracle; oracle.build(sanitize=True)'
rt=$(/opt/rocm/llvm/bin/clang -print-file-name=libclang_rt.asan-x86_64.so)
export WD_LIB_PATH="$PWD/paper_0911_3191_amd/libwdslash_san.so"
export WD_ORACLE_LIB="$PWD/oracle/libwdoracle_san.so"
export ASAN_OPTIONS=detect_leaks=0:abort_on_error=1
export UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1
LD_PRELOAD="$rt" python -m pytest tests -m "not gpu" -q -p no:cacheprovider "$@"
