#pragma once
#include "../../hipemu.hpp"
