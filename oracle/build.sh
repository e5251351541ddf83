#!/bin/sh
# Builds the oracle (test infrastructure) as liboracle.so beside this script.
# -ffp-contract=off: no fused multiply-add unless written as fma().
#   sh oracle/build.sh            the oracle the tests use
#   sh oracle/build.sh sanitize   liboracle_san.so: the same sources under
#                                 AddressSanitizer and UndefinedBehaviorSanitizer
#                                 (host code only; load with libasan preloaded)
set -e
here=$(cd "$(dirname "$0")" && pwd)
if [ "$1" = "sanitize" ]; then
  g++ -std=c++17 -O1 -g -fno-omit-frame-pointer -ffp-contract=off -fPIC -shared -pthread -Wall -Wextra \
      -Wno-unused-parameter -fsanitize=address,undefined -fno-sanitize-recover=undefined \
      -o "$here/liboracle_san.so" "$here/ref_api.cpp"
else
  g++ -std=c++17 -O2 -ffp-contract=off -fPIC -shared -pthread -Wall -Wextra -Wno-unused-parameter \
      -o "$here/liboracle.so" "$here/ref_api.cpp"
fi
