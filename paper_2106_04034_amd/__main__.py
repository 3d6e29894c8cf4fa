"""Command line in the manner of the paper's program (Section 3.3):

    python -m paper_2106_04034_amd -train_file train.txt -test_file test.txt

reads the fitness cases (features in columns, target last), runs GSGP on the
GPU and writes two text files, the best train fitness of every generation and
the test fitness of that individual.  The parameters the paper keeps in a
configuration file are options here.
"""
from __future__ import annotations

import argparse
import sys

from . import cases, gsgp


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2106_04034_amd", description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("-train_file", required=True)
    ap.add_argument("-test_file", default=None)
    ap.add_argument("--population", type=int, default=1024)
    ap.add_argument("--pool", type=int, default=1024)
    ap.add_argument("--genome-length", type=int, default=127)
    ap.add_argument("--generations", type=int, default=100)
    ap.add_argument("--tournament-size", type=int, default=4, help="0: mutate every individual (paper loop)")
    ap.add_argument("--p-crossover", type=float, default=0.5)
    ap.add_argument("--mutation-step", type=float, default=0.1)
    ap.add_argument("--random-step", action="store_true", help="draw each mutation step in [0, step)")
    ap.add_argument("--precision", choices=sorted(gsgp.PRECISIONS), default="fp32")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out-train", default="fitness_train.txt")
    ap.add_argument("--out-test", default="fitness_test.txt")
    a = ap.parse_args(argv)
    data = cases.read_dataset(a.train_file, a.test_file)
    s = gsgp.Settings(pop_size=a.population, pool_size=a.pool, genome_len=a.genome_length,
                      n_generations_max=a.generations, tournament_size=a.tournament_size,
                      p_crossover=0.0 if a.tournament_size == 0 else a.p_crossover,
                      mutation_step=a.mutation_step, ms_random=1 if a.random_step else 0,
                      precision=gsgp.PRECISIONS[a.precision], seed=a.seed)
    R = gsgp.Runner(s, [data])
    R.eval_population()
    R.generation(a.generations, stats=False)
    stats = R.stats(0, 0, a.generations + 1)
    R.close()
    cases.write_fitness_files(stats, a.out_train, a.out_test)
    best = stats[-1]
    print(f"generation {a.generations}: best train RMSE {best['best_train_rmse']:.6g}, "
          f"its test RMSE {best['best_test_rmse']:.6g} (individual {best['best_index']})")
    return 0


if __name__ == "__main__":
    sys.exit(main())
