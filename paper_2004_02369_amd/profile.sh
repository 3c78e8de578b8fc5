#!/bin/bash
# rocprofv3 passes over the benchmark's timed launch (bench.py --no-extras):
# kernel trace, HBM-side bytes (FETCH_SIZE, WRITE_SIZE, one counter per pass),
# issue counters (SQ), texture-unit and L1->L2 counters (TA/TCP), and the
# plain-copy calibration of FETCH_SIZE / WRITE_SIZE.  Raw output goes to
# gpurun_out/prof_<pass>/; summarise with `python -m paper_2004_02369_amd.profsum`.
#   bash paper_2004_02369_amd/profile.sh [passes...]   (default: all)
set -o pipefail
cd "$(dirname "$0")/.." || exit 1
export TMPDIR=/tmp
BENCH=(python3 bench.py --steps 2 --warmup 0 --no-cpu-baseline --no-extras)
passes=("$@")
[ ${#passes[@]} -eq 0 ] && passes=(kt fetch write sq ta cfetch cwrite)
for p in "${passes[@]}"; do
  echo "[profile] pass $p"
  case $p in
    kt) timeout -k 10 400 rocprofv3 --kernel-trace --stats -d gpurun_out/prof_kt -o kt --output-format csv -- "${BENCH[@]}" ;;
    fetch) timeout -s KILL 400 rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof_fetch -o f --output-format csv -- "${BENCH[@]}" ;;
    write) timeout -s KILL 400 rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof_write -o w --output-format csv -- "${BENCH[@]}" ;;
    sq) timeout -s KILL 400 rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_ANY SQ_WAVE_CYCLES SQ_BUSY_CYCLES -d gpurun_out/prof_sq -o sq --output-format csv -- "${BENCH[@]}" ;;
    ta) timeout -s KILL 400 rocprofv3 --pmc TA_BUSY_avr TA_BUSY_max TCP_TCC_READ_REQ_sum -d gpurun_out/prof_ta -o ta --output-format csv -- "${BENCH[@]}" ;;
    cfetch) timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof_cfetch -o cf --output-format csv -- python3 bench.py --calibrate-copy 512 ;;
    cwrite) timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof_cwrite -o cw --output-format csv -- python3 bench.py --calibrate-copy 512 ;;
    *) echo "unknown pass $p"; exit 2 ;;
  esac
  rc=$?
  if [ $rc -ne 0 ]; then echo "[profile] pass $p failed rc=$rc"; exit $rc; fi
done
