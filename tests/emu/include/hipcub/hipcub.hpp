#pragma once
#include "../../hipemu_cub.hpp"
