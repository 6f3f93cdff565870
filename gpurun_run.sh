set -o pipefail
mkdir -p gpurun_out
echo "[gpu] full GPU suite"
timeout -k 10 1200 python -u -m pytest tests -m gpu -x -v -s --timeout 300 --timeout-method thread > gpurun_out/pytest_all.log 2>&1
rc=$?; grep -E "separable|PASS|FAIL|Error|passed|failed" gpurun_out/pytest_all.log | tail -12; [ $rc -eq 0 ] || exit $rc
for W in sn_core spheroid binary; do
echo "[gpu] bench $W"
timeout -k 10 600 python -u bench.py --workload $W --steps 10 --warmup 2 --no-cpu-baseline > gpurun_out/bench6_$W.json 2> gpurun_out/bench6_$W.err
rc=$?; grep "\[bench\] fp64" gpurun_out/bench6_$W.err | tail -3; [ $rc -eq 0 ] || exit $rc
done
