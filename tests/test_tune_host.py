"""Host logic of the autotuner (no GPU): deriving the thread-group form
thresholds from the best form of each batch-size interval."""
from paper_2309_09025_amd import fhesnn as F
from paper_2309_09025_amd import tune


def test_measured_order_gives_one_interval_per_form():
    assert tune.thresholds_from_best(["rows", "paired", "two", "one"], 256) == (256, 512, 768)


def test_runs_of_one_form_extend_its_threshold():
    assert tune.thresholds_from_best(["rows", "paired", "paired", "two"], 256) == (256, 768, 1024)
    assert tune.thresholds_from_best(["rows", "rows", "one", "one"], 100) == (200, 200, 200)


def test_an_earlier_form_inside_a_later_run_does_not_end_it():
    # the library checks the forms in order, so an interval whose best form
    # is an earlier one is served by the later form's threshold range
    assert tune.thresholds_from_best(["paired", "rows", "two", "one"], 256) == (0, 512, 768)


def test_no_intervals_disable_every_small_batch_form():
    assert tune.thresholds_from_best([], 256) == (0, 0, 0)


def test_committed_cache_is_well_formed():
    """Every cached variant choice names an existing variant and was the
    fastest of the timings of all variants of its ring degree; every cached form list names known forms."""
    import json
    with open(tune.CACHE) as fh:
        cache = json.load(fh)
    assert cache
    for key, rec in cache.items():
        if "|groups|" in key:
            assert rec["best"] and set(rec["best"]) <= set(tune.FORMS), key
            for jobs, ms in rec["ms"].items():
                assert rec["best"][sorted(map(int, rec["ms"])).index(int(jobs))] == \
                    min(ms, key=ms.get), (key, jobs)
        else:
            ms = {int(v): t for v, t in rec["ms"].items()}
            N = int(key.split("|N=")[1].split("|")[0])
            # every variant of the ring degree was timed (a host query of the library)
            assert sorted(ms) == list(range(F.br_variants(N))), key
            assert rec["variant"] == min(ms, key=ms.get), key
