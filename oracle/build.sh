#!/bin/sh
# Builds the CPU oracle (test infrastructure only) as oracle/liblpf_oracle.so.
set -e
cd "$(dirname "$0")"
gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC -Wall -Wextra \
    -o liblpf_oracle.so lpf_oracle.c -lm
