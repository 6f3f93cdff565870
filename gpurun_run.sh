set -o pipefail
mkdir -p gpurun_out
echo "[gpu] pytest precision start"
timeout -k 10 900 python -u -m pytest tests/test_gpu_precision.py -x -v -s --timeout 300 --timeout-method thread > gpurun_out/pytest_prec.log 2>&1
rc=$?; grep -E "max rel err|variant|PASS|FAIL|Error|error" gpurun_out/pytest_prec.log | tail -40; tail -5 gpurun_out/pytest_prec.log; [ $rc -eq 0 ] || exit $rc
for p in bf16x3 fp16x2 fp32; do
echo "[gpu] bench binary $p"
timeout -k 10 600 python -u bench.py --workload binary --precision $p --steps 5 --warmup 2 --no-cpu-baseline --no-check > gpurun_out/bench_bin_$p.json 2> gpurun_out/bench_bin_$p.err
rc=$?; tail -4 gpurun_out/bench_bin_$p.err; cat gpurun_out/bench_bin_$p.json; [ $rc -eq 0 ] || exit $rc
done
