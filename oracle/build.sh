#!/bin/sh
# Builds the oracle (test infrastructure) as a shared library with the
# floating-point environment the format fixes: no contraction, no fast-math.
set -e
cd "$(dirname "$0")"
gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off -fno-fast-math -Wall -Wextra -o libfzo.so fzo.c -lm
