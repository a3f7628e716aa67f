#!/bin/sh
# Builds the CPU oracle (test infrastructure only) into oracle/liborc.so.
set -e
cd "$(dirname "$0")"
g++ -O2 -std=c++17 -fopenmp -fPIC -shared -Wall -Wno-unknown-pragmas \
    orc_dirac.cpp orc_solve.cpp orc_net.cpp orc_force.cpp orc_api.cpp -o liborc.so.tmp
mv liborc.so.tmp liborc.so
