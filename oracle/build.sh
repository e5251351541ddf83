#!/bin/sh
# Builds the oracle (test infrastructure) as liboracle.so beside this script.
# -ffp-contract=off: no fused multiply-add unless written as fma().
set -e
here=$(cd "$(dirname "$0")" && pwd)
g++ -std=c++17 -O2 -ffp-contract=off -fPIC -shared -pthread -Wall -Wextra -Wno-unused-parameter \
    -o "$here/liboracle.so" "$here/ref_api.cpp"
