#!/bin/sh
# Builds the CPU oracle (test infrastructure only) into oracle/liborc.so.
# SANITIZE=1 builds it with AddressSanitizer and UndefinedBehaviorSanitizer (load
# it with the ASan runtime preloaded, e.g.
#   LD_PRELOAD=$(gcc -print-file-name=libasan.so) ASAN_OPTIONS=detect_leaks=0 python -m pytest ...).
set -e
cd "$(dirname "$0")"
if [ "${SANITIZE:-0}" = "1" ]; then
  EXTRA="-fsanitize=address,undefined -fno-omit-frame-pointer -fno-sanitize-recover=undefined"
else
  EXTRA=""
fi
g++ -O2 -std=c++17 -fopenmp -fPIC -shared -Wall -Wno-unknown-pragmas $EXTRA \
    orc_dirac.cpp orc_solve.cpp orc_net.cpp orc_force.cpp orc_api.cpp -o liborc.so.tmp
mv liborc.so.tmp liborc.so
