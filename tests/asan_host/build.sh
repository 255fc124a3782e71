# AddressSanitizer + UBSan build of libmplb's host code (the device code is
# built as usual), linked into driver.cpp, which calls every C-ABI entry point
# with valid arguments and on its error paths.  Builds on a machine without a
# GPU; the binary runs where one is present:
#
#   bash tests/asan_host/build.sh
#   ASAN_OPTIONS=detect_leaks=1:protect_shadow_gap=0 \
#   LSAN_OPTIONS=suppressions=tests/asan_host/lsan.supp tests/asan_host/_build/driver
#
# (lsan.supp suppresses the HIP runtime's own allocations that live until
# exit; protect_shadow_gap=0 leaves the shadow gap to the GPU driver's
# mappings.)  It prints "ok: 0 failed expectations" and exits 0 when every
# call returned what it should and no sanitizer reported an error.
set -e
R="$(cd "$(dirname "$0")/../.." && pwd)"
D="$R/tests/asan_host"
mkdir -p "$D/_build"
F="--offload-arch=gfx950 -O1 -g -std=c++17 -Xclang -target-feature -Xclang -packed-fp32-ops -I $R/include -I $R/paper_1507_07294_amd/csrc -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer -Wno-unused-command-line-argument"
/opt/rocm/bin/hipcc $F -c "$D/driver.cpp" -o "$D/_build/driver.o"
/opt/rocm/bin/hipcc $F -c "$R/paper_1507_07294_amd/csrc/mplb.cpp" -o "$D/_build/mplb.o"
/opt/rocm/bin/hipcc $F -c -x hip "$R/paper_1507_07294_amd/csrc/fused.hip" -o "$D/_build/fused.o"
/opt/rocm/bin/hipcc $F -c -x hip "$R/paper_1507_07294_amd/csrc/kernels.hip" -o "$D/_build/kernels.o"
/opt/rocm/llvm/bin/clang++ -fsanitize=address,undefined "$D"/_build/*.o -L/opt/rocm/lib -lamdhip64 \
    -Wl,-rpath,/opt/rocm/lib -o "$D/_build/driver"
rm -f "$D"/_build/*.o
