"""Host logic of the profile summaries: rocprofv3 kernel names map to the
timing kinds the library records live, and a counter summary written from
FETCH_SIZE / WRITE_SIZE files reads back with the calibration applied."""
import csv

from paper_1809_07444_amd import _capi as C
from paper_1809_07444_amd import profiling as P

# Names as rocprofv3 prints them for kernels built from these sources.
TRACE_NAMES = {
    "void dsoar::doall_kernel<dsoar::(anonymous namespace)::AlivePrep>(dsoar::DevHeap, unsigned int, "
    "unsigned int const*, unsigned long const*, unsigned int const*, "
    "dsoar::(anonymous namespace)::AlivePrep::Args)": "gol_alive_prep",
    "void dsoar::doall_kernel<dsoar::(anonymous namespace)::BodyForce>(dsoar::DevHeap, unsigned int, "
    "unsigned int const*, unsigned long const*, unsigned int const*, "
    "dsoar::(anonymous namespace)::BodyForce::Args)": "collide_force",
    "void dsoar::doall2_kernel<dsoar::(anonymous namespace)::AliveUpdate, dsoar::(anonymous namespace)::"
    "CandUpdate>(dsoar::DevHeap, unsigned int, unsigned int const*, unsigned long const*, unsigned int const*, "
    "dsoar::(anonymous namespace)::AliveUpdate::Args, unsigned int, unsigned int const*, unsigned long const*, "
    "unsigned int const*, dsoar::(anonymous namespace)::CandUpdate::Args)": "gol_update",
    "void dsoar::(anonymous namespace)::enumerate_kernel<1u>(dsoar::DevHeap, unsigned int, dsoar::EnumOut)":
        "enumerate",
    "void dsoar::(anonymous namespace)::enumerate_kernel<8u>(dsoar::DevHeap, unsigned int, dsoar::EnumOut)":
        "enumerate",
    "dsoar::(anonymous namespace)::entry_kernel(dsoar::DevHeap, dsoar::(anonymous namespace)::Road)":
        "traffic_entry",
    "dsoar::(anonymous namespace)::tick_kernel(dsoar::(anonymous namespace)::Sea)": "wator_tick",
    "dsoar::(anonymous namespace)::micro_create_kernel(dsoar::DevHeap, unsigned int, unsigned int, "
    "unsigned int, unsigned int, float const*, float const*)": "micro_create",
    "dsoar::(anonymous namespace)::gol_init_kernel(dsoar::DevHeap, dsoar::(anonymous namespace)::World, "
    "unsigned int, unsigned int, unsigned char const*)": "gol_init",
    "dsoar::(anonymous namespace)::regrow_kernel(dsoar::(anonymous namespace)::Grid)": "sugar_regrow",
    "dsoar::(anonymous namespace)::init_heap_kernel(dsoar::DevHeap, unsigned long)": None,
    # Instances per bitmap container width.
    "void dsoar::doall_kernel<dsoar::(anonymous namespace)::AlivePrep, 6u>(dsoar::DevHeapW<6u>, unsigned int, "
    "unsigned int const*, unsigned long const*, unsigned int const*, "
    "dsoar::(anonymous namespace)::AlivePrep::Args)": "gol_alive_prep",
    "void dsoar::doall2_kernel<dsoar::(anonymous namespace)::AliveUpdate, dsoar::(anonymous namespace)::"
    "CandUpdate, 5u>(dsoar::DevHeapW<5u>, unsigned int, unsigned int const*, unsigned long const*, "
    "unsigned int const*, dsoar::(anonymous namespace)::AliveUpdate::Args, unsigned int, unsigned int const*, "
    "unsigned long const*, unsigned int const*, dsoar::(anonymous namespace)::CandUpdate::Args)": "gol_update",
    "void dsoar::(anonymous namespace)::enumerate_kernel<8u, 6u>(dsoar::DevHeapW<6u>, unsigned int, "
    "dsoar::EnumOut)": "enumerate",
    # Do-alls instantiated for large heaps (more resident wavefronts) or not.
    "void dsoar::doall2_kernel<dsoar::(anonymous namespace)::AliveUpdate, dsoar::(anonymous namespace)::"
    "CandUpdate, 6u, true>(dsoar::DevHeapW<6u>, unsigned int, unsigned int const*, unsigned long const*, "
    "unsigned int const*, dsoar::(anonymous namespace)::AliveUpdate::Args, unsigned int, unsigned int const*, "
    "unsigned long const*, unsigned int const*, dsoar::(anonymous namespace)::CandUpdate::Args)": "gol_update",
    "void dsoar::doall_kernel<dsoar::(anonymous namespace)::Eat, 6u, false>(dsoar::DevHeapW<6u>, unsigned int, "
    "unsigned int const*, unsigned long const*, unsigned int const*, "
    "dsoar::(anonymous namespace)::Eat::Args)": "sugar_eat",
    "void dsoar::(anonymous namespace)::gol_init_kernel<6u>(dsoar::DevHeapW<6u>, "
    "dsoar::(anonymous namespace)::World, unsigned int, unsigned int, unsigned char const*)": "gol_init",
    "void dsoar::(anonymous namespace)::entry_kernel<5u>(dsoar::DevHeapW<5u>, dsoar::(anonymous namespace)::Road)":
        "traffic_entry",
    "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<int>, "
    "std::array<char*, 2ul> >(int, at::native::CUDAFunctorOnSelf_add<int>, std::array<char*, 2ul>)":
        "calibration",
    "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<int>, std::array<char*, 1ul> >"
    "(int, at::native::FillFunctor<int>, std::array<char*, 1ul>)": None,
}


def test_trace_names_map_to_kinds():
    for name, kind in TRACE_NAMES.items():
        assert P.kernel_kind(name) == kind, name


def test_every_traced_kind_is_a_live_timing_kind():
    # The summaries and the live per-launch timing must name kernels alike,
    # or the benchmark could not match a traced kernel with its live figure.
    live = set(C.KIND_NAMES.values())
    traced = set(P.METHOD_KIND.values()) | set(P.METHOD2_KIND.values()) | {k for _, _, k in P.PLAIN_KIND}
    assert traced <= live
    assert "enumerate" in live


def _counter_csv(path, rows, counter):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_summary_round_trip_with_calibration(tmp_path):
    add = [n for n, k in TRACE_NAMES.items() if k == "calibration"][0]
    prep = [n for n, k in TRACE_NAMES.items() if k == "gol_alive_prep"][0]
    other = [n for n, k in TRACE_NAMES.items() if k is None][0]
    cal = P.CAL_BYTES_KIB
    # The counters read half the calibration copy's bytes on fetch and all of
    # them on write: the factors are 2 and 1.
    _counter_csv(tmp_path / "f.csv", [(add, cal / 2), (prep, 100.0), (prep, 300.0), (other, 7.0)], "FETCH_SIZE")
    _counter_csv(tmp_path / "w.csv", [(add, cal), (prep, 50.0), (prep, 50.0), (other, 7.0)], "WRITE_SIZE")
    s = P.summarize(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert abs(s["fetch_factor"] - 2.0) < 1e-12 and abs(s["write_factor"] - 1.0) < 1e-12
    k = s["kernels"]["gol_alive_prep"]
    assert k["dispatches"] == 2 and k["fetch_kib"] == 200.0 and k["write_kib"] == 50.0
    assert k["bytes"] == (200.0 * 2 + 50.0) * 1024
    assert set(s["kernels"]) == {"gol_alive_prep"}
    out = tmp_path / "traffic_x.txt"
    P.write_summary(str(out), "x", s, "cmd", "abcd")
    back = P.read_summary(str(out))
    assert back["source_hash"] == "abcd" and back["kernels"] == {"gol_alive_prep": (200.0 * 2 + 50.0) * 1024}
    assert P.read_summary(str(tmp_path / "missing.txt")) is None


def test_kernel_kinds_of_the_sources_are_named_once():
    # The device code tags each timed launch with a kind number; the binding
    # names them.  Every number in the sources has a name, none is used twice,
    # and no name is left without a kernel.
    import glob
    import os
    import re
    csrc = os.path.join(os.path.dirname(C.__file__), "csrc")
    nums = []
    for path in sorted(glob.glob(os.path.join(csrc, "*.h*p*"))):
        with open(path) as fh:
            nums += [int(n) for n in re.findall(r"\bkKind\w* = (\d+)", fh.read())]
    assert len(nums) == len(set(nums))
    assert set(nums) == set(C.KIND_NAMES)
    assert len(set(C.KIND_NAMES.values())) == len(C.KIND_NAMES)
