#!/bin/bash
# Builds tests/helpers/abi_asan_driver (see that file): the library's sources
# with AddressSanitizer and UndefinedBehaviorSanitizer on host code only (a
# report ends the run), the driver and the oracle with them too, linked into
# one executable next to this script.
set -e
H=$(cd "$(dirname "$0")" && pwd)
R=$(cd "$H/../.." && pwd)
O=$(mktemp -d)
F="-O1 -g -std=c++17 -fPIC --offload-arch=gfx950 -ffp-contract=off -fno-fast-math -Xclang -target-feature -Xclang -packed-fp32-ops -pthread -fno-omit-frame-pointer"
for f in rdos_kernels.hip rdos_api.cpp rdos_engine.cpp; do
  /opt/rocm/bin/hipcc $F -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all -x hip -c "$R/paper_1512_03126_amd/csrc/$f" -o "$O/${f%.*}.o"
done
/opt/rocm/llvm/bin/clang -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all -fno-omit-frame-pointer -ffp-contract=off -I "$R/include" -I "$R/oracle" -c "$H/abi_asan_driver.c" -o "$O/drv.o"
/opt/rocm/llvm/bin/clang -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all -fno-omit-frame-pointer -ffp-contract=off -std=c11 -I "$R/oracle" -c "$R/oracle/oracle.c" -o "$O/oracle.o"
/opt/rocm/bin/hipcc --offload-arch=gfx950 -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -pthread -o "$H/abi_asan_driver" \
    "$O/drv.o" "$O/oracle.o" "$O/rdos_kernels.o" "$O/rdos_api.o" "$O/rdos_engine.o"
rm -rf "$O"
echo "$H/abi_asan_driver"
