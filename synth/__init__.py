from . import problem, generate  # noqa: F401
