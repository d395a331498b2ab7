#!/bin/bash
# Builds libdeltamic.so (and the ALU probe library libdmprobe.so) for gfx950
# in this directory's parent package folder.
set -euo pipefail
HERE="$(cd "$(dirname "${BASH_SOURCE[0]}")" && pwd)"
OUT="${1:-$HERE/../libdeltamic.so}"
ROCM="${ROCM_PATH:-/opt/rocm}"
FLAGS=(-O3 -std=c++17 -fPIC --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
       -I"$HERE/../../include" -I"$ROCM/include")
TMP="$(mktemp -d)"
trap 'rm -rf "$TMP"' EXIT
"$ROCM/bin/hipcc" "${FLAGS[@]}" -c "$HERE/dm_kernels.hip" -o "$TMP/dm_kernels.o"
"$ROCM/bin/hipcc" "${FLAGS[@]}" -c "$HERE/dm_precond.hip" -o "$TMP/dm_precond.o"
"$ROCM/bin/hipcc" "${FLAGS[@]}" -c "$HERE/dm_scratch.hip" -o "$TMP/dm_scratch.o"
"$ROCM/bin/hipcc" "${FLAGS[@]}" -c "$HERE/dm_host.cpp" -o "$TMP/dm_host.o"
"$ROCM/bin/hipcc" "${FLAGS[@]}" -c "$HERE/dm_topo.cpp" -o "$TMP/dm_topo.o"
"$ROCM/bin/hipcc" -shared --offload-arch=gfx950 -o "$OUT.tmp" "$TMP/dm_kernels.o" "$TMP/dm_precond.o" "$TMP/dm_scratch.o" "$TMP/dm_host.o" "$TMP/dm_topo.o" \
  -L"$ROCM/lib" -lrocfft -Wl,-rpath,"$ROCM/lib"
mv -f "$OUT.tmp" "$OUT"
echo "built $OUT"
# ALU throughput probes used by the benchmark to price the sweeps (own library)
PROBE="$(dirname "$OUT")/libdmprobe.so"
"$ROCM/bin/hipcc" "${FLAGS[@]}" -shared -o "$PROBE.tmp" "$HERE/dm_probe.hip"
mv -f "$PROBE.tmp" "$PROBE"
echo "built $PROBE"
