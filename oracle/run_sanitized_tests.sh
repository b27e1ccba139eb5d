#!/bin/sh
# The CPU test suite (-m "not gpu") against an AddressSanitizer +
# UndefinedBehaviorSanitizer build of the oracle (oracle/liboracle_gs_san.so).
# The sanitizer runtimes are preloaded into the Python process; leak checking
# is off (the interpreter itself keeps memory until exit).  Extra arguments go
# to pytest.
set -e
ROOT=$(cd "$(dirname "$0")/.." && pwd)
cd "$ROOT"
GS_ORACLE_SANITIZE=1 python -c "from oracle import gs_oracle; print(gs_oracle.build())"
ASAN_RT=$(gcc -print-file-name=libasan.so)
UBSAN_RT=$(gcc -print-file-name=libubsan.so)
LD_PRELOAD="$ASAN_RT $UBSAN_RT" \
ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 \
UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
GS_ORACLE_SANITIZE=1 \
python -m pytest tests -q -m "not gpu" "$@"
